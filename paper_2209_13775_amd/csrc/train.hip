// train.hip -- fused training step of the Fourier-feature MLP surrogate:
// one Adam step on the mean squared error of the predicted window
// displacement, in four launches.
//
//   train_fwd_kernel     per 128 samples: features, the four hidden layers on
//                        MFMA with the activations resident in LDS, head, MSE
//                        gradient; stores gelu'(z) of every hidden layer and
//                        the layer inputs for the weight gradients, and the
//                        head's gradient and the loss as per-tile partials
//   train_bwd_kernel     per 128 samples: back-propagation through the hidden
//                        layers on MFMA (activation gradients in LDS); stores
//                        dz of every layer
//   train_wgrad_kernel   per chunk of 2048 samples: dW_l = h_l^T dz_l for the
//                        four layers (MFMA, fragments loaded straight from the
//                        stored layouts), the bias sums of dz_l, and the head
//                        partials of the chunk's tiles summed
//   train_update_kernel  chunk partials summed in order, Adam, and the BF16
//                        copies of the updated hidden matrices
//
// Layouts in the workspace (batch padded to whole 128-sample tiles, Bp):
//   fragment layout (gelu'(z)): per tile and layer, the 128 x 256 values in
//     the order the product's accumulators hold them -- wave w, output block
//     j, sample block i, lane, 4 consecutive outputs -- so that each lane
//     stores and later loads 8 contiguous bytes;
//   T8 layout (layer inputs h_l, gradients dz_l): [Bp/8][K][8], eight
//     consecutive samples of one column contiguous, which is the reduction
//     operand of the weight-gradient MFMA (8 consecutive reduction indices
//     per lane).
// Every sum runs in a fixed order, so a step is bit-reproducible.

#include "lcs_internal.h"
#include "device_common.h"

namespace lcs {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kTS = 128;                    // samples per tile
constexpr int kTT = 512;                    // threads of the forward and backward kernels
constexpr int kTW = kTT / 64;               // their waves: wave w owns outputs kNJ*16*w ..
constexpr int kNJ = kMlpWidth / (16 * kTW); // 16-wide output blocks per wave
static_assert(kNJ * 16 * kTW == kMlpWidth && kTT >= 2 * kTS && kTT >= kMlpWidth,
              "the output blocks, the head's two threads per sample and its gradient's thread per "
              "input must fit the workgroup");
constexpr int kStr = kMlpWidth + 8;         // BF16 per LDS activation row (16-byte aligned rows)
constexpr long long kFragTile = (long long)kTS * kMlpWidth;   // BF16 per tile and layer
constexpr int kWgradTiles = 2 + 4 * (kMlpHidden - 1);          // 128 x 128 weight-gradient tiles

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// four floats rounded to BF16 (nearest even), packed into 8 bytes
__device__ __forceinline__ uint2 pack4(float a, float b, float c, float d)
{
    const bf16x2 lo = __builtin_convertvector((f32x2){a, b}, bf16x2);
    const bf16x2 hi = __builtin_convertvector((f32x2){c, d}, bf16x2);
    return make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
}

__device__ __forceinline__ void unpack4(uint2 v, float *o)
{
    o[0] = __uint_as_float(v.x << 16);
    o[1] = __uint_as_float(v.x & 0xffff0000u);
    o[2] = __uint_as_float(v.y << 16);
    o[3] = __uint_as_float(v.y & 0xffff0000u);
}

// tanh-form GELU and its derivative from one logistic value:
// gelu(z) = z s with s = 1 / (1 + exp(-2u)), u = sqrt(2/pi) (z + 0.044715 z^3);
// gelu'(z) = s + z s (1 - s) du2/dz with du2/dz = 2 sqrt(2/pi) (1 + 3 * 0.044715 z^2).
// -2u log2(e) is folded into z (A + B z^2) ahead of a base-2 exponential.
__device__ __forceinline__ void gelu_pair(float z, float &h, float &d)
{
    constexpr float A = -2.3022082f;    // -2 log2(e) sqrt(2/pi)
    constexpr float B = -0.10294324f;   // A * 0.044715
    constexpr float C1 = 1.5957691f;    // 2 sqrt(2/pi)
    constexpr float C2 = 0.21406445f;   // 6 * 0.044715 sqrt(2/pi)
    const float z2 = z * z;
    const float s = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z * fmaf(B, z2, A)));
    h = z * s;
    d = s * fmaf(z * (1.0f - s), fmaf(C2, z2, C1), 1.0f);
}

// One layer's product for the tile, transposed: out^T[n][m] = sum_k A[n][k] act[m][k]
// with A from global memory (BF16, N x K, row-major or -- FRAG -- in fragment
// order, where a wave's fragment is one contiguous 1 KiB) and the activations
// in LDS; wave w owns outputs 32w .. 32w+31.  acc must hold the starting
// values.  The next 32-wide slice of A is loaded while the current one's
// products run.
template <int K, bool FRAG>
__device__ __forceinline__ void tile_product(const uint16_t *__restrict__ Arows, const uint16_t *act,
                                             f32x4 (&acc)[8][kNJ], int wave, int lane)
{
    static_assert(K % 64 == 0, "K must be a multiple of 64");
    const int ko = 8 * (lane / 16);
    // per output block j, the lane's 32-bit element offset at k = 0 (a matrix
    // holds at most 256 x 256 values); a k-slice adds a wave-uniform step
    uint32_t base[kNJ];
#pragma unroll
    for (int j = 0; j < kNJ; ++j)
        base[j] = FRAG ? (uint32_t)((wave * kNJ + j) * (K / 32) * 512 + lane * 8)
                       : (uint32_t)((wave * 16 * kNJ + 16 * j + lane % 16) * K + ko);
    auto load_a = [&](int kk, bf16x8 *w) {
#pragma unroll
        for (int j = 0; j < kNJ; ++j)
            w[j] = *reinterpret_cast<const bf16x8 *>(Arows + base[j] + (FRAG ? (uint32_t)(kk / 32 * 512)
                                                                          : (uint32_t)kk));
    };
    auto slice = [&](int kk, const bf16x8 *w) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const bf16x8 xb = *reinterpret_cast<const bf16x8 *>(&act[(16 * i + lane % 16) * kStr + kk + ko]);
#pragma unroll
            for (int j = 0; j < kNJ; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[j], xb, acc[i][j], 0, 0, 0);
        }
    };
    bf16x8 wa[kNJ], wb[kNJ];
    load_a(0, wa);
    for (int kk = 0; kk < K; kk += 64) {
        load_a(kk + 32, wb);
        __builtin_amdgcn_sched_barrier(0);
        slice(kk, wa);
        if (kk + 64 < K) load_a(kk + 64, wa);
        __builtin_amdgcn_sched_barrier(0);
        slice(kk + 32, wb);
    }
}

// The tile's LDS activations (128 x K) written to a T8 array of K columns;
// thread t takes column t % K.  The stores are non-temporal: a T8 array is
// read back only by a later kernel (the weight gradients); streamed past the
// caches, the backward kernel went 81 -> 65 us and the weight gradients
// 93 -> 87 us per step for the same counted HBM bytes (non-temporal loads in
// the weight gradients, which read each element twice, were slower).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <int K>
__device__ __forceinline__ void store_t8(const uint16_t *act, uint16_t *__restrict__ out, long long tile,
                                         int tid)
{
    const int k = tid % K;
    for (int g = tid / K; g < kTS / 8; g += kTT / K) {
        uint16_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = act[(8 * g + q) * kStr + k];
        const u32x4 w = {(uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16),
                         (uint32_t)v[4] | ((uint32_t)v[5] << 16), (uint32_t)v[6] | ((uint32_t)v[7] << 16)};
        __builtin_nontemporal_store(w, reinterpret_cast<u32x4 *>(out + ((tile * (kTS / 8) + g) * K + k) * 8));
    }
}

// A lane's 4 gelu' values of one block, loaded non-temporally: each is read
// once, by the backward kernel (228 against 231 us per step).
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void load_frag4(const uint16_t *p, float *o)
{
    const u32x2 q = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p));
    unpack4(make_uint2(q.x, q.y), o);
}

// offset (BF16 elements) of a lane's 4 values of block (i, j) in the fragment layout
__device__ __forceinline__ long long frag_off(long long tile, int wave, int j, int i, int lane)
{
    return tile * kFragTile + ((long long)((wave * kNJ + j) * 8 + i) * 64 + lane) * 4;
}

__global__ __launch_bounds__(kTT, 4) void train_fwd_kernel(TrainArgs A)
{
    __shared__ __attribute__((aligned(16))) uint16_t act[kTS * kStr];
    __shared__ float xs[4][kTS];
    __shared__ float yp[3][kTS];
    __shared__ float dys[3][kTS];
    __shared__ double lsum[kTS];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const long long tile = blockIdx.x;
    const long long m0 = tile * kTS;
    const MlpDev &P = A.P;
    if (tid < kTS) {
        const long long m = min(m0 + tid, A.B - 1);     // padding rows repeat the last sample
#pragma unroll
        for (int a = 0; a < 4; ++a) xs[a][tid] = A.xt[a * A.ld + m];
    }
    __syncthreads();
    // Fourier features, thread -> (sample m, frequency f), f fastest; phase in
    // revolutions reduced exactly to [-1/2, 1/2], hardware sine and cosine
    for (int idx = tid; idx < kTS * kMlpFreq; idx += kTT) {
        const int m = idx / kMlpFreq, f = idx % kMlpFreq;
        const float *b = P.freq + 4 * f;
        float rev = 0.0f;
#pragma unroll
        for (int a = 0; a < 4; ++a) rev += b[a] * ((xs[a][m] - P.in_shift[a]) * P.in_scale[a]);
        const float r = rev - rintf(rev);
        act[m * kStr + f] = __builtin_bit_cast(uint16_t, (__bf16)__builtin_amdgcn_cosf(r));
        act[m * kStr + kMlpFreq + f] = __builtin_bit_cast(uint16_t, (__bf16)__builtin_amdgcn_sinf(r));
    }
    __syncthreads();
    store_t8<kMlpFeat>(act, A.ht[0], tile, tid);
    for (int l = 0; l < kMlpHidden; ++l) {
        const float *bias = P.params + mlp_off_b(l);
        f32x4 acc[8][kNJ];
#pragma unroll
        for (int j = 0; j < kNJ; ++j) {
            const int n0 = wave * 16 * kNJ + 16 * j + 4 * (lane / 16);
            const f32x4 b4 = (f32x4){bias[n0], bias[n0 + 1], bias[n0 + 2], bias[n0 + 3]};
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i][j] = b4;
        }
        // W_l^T ([out][in] copy, fragment order)
        const uint16_t *Wt = P.wbf + mlp_off_bf16(l) + (long long)mlp_in_width(l) * kMlpWidth;
        if (l == 0) tile_product<kMlpFeat, true>(Wt, act, acc, wave, lane);
        else tile_product<kMlpWidth, true>(Wt, act, acc, wave, lane);
        __syncthreads();   // every wave has read the layer input
        uint16_t *dl = A.dgelu[l];
#pragma unroll
        for (int j = 0; j < kNJ; ++j) {
            const int n0 = wave * 16 * kNJ + 16 * j + 4 * (lane / 16);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                float h[4], d[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) gelu_pair(acc[i][j][e], h[e], d[e]);
                *reinterpret_cast<uint2 *>(&act[(16 * i + lane % 16) * kStr + n0]) =
                    pack4(h[0], h[1], h[2], h[3]);
                *reinterpret_cast<uint2 *>(dl + frag_off(tile, wave, j, i, lane)) =
                    pack4(d[0], d[1], d[2], d[3]);
            }
        }
        __syncthreads();
        if (l + 1 < kMlpHidden) store_t8<kMlpWidth>(act, A.ht[l + 1], tile, tid);
    }
    // head (FP32): two threads per sample (waves 0-3), halves of the 256 inputs
    // uniform per wave so the head weights are scalar loads
    const float *Wh = P.params + kOffWh;
    const float *bh = P.params + kOffBh;
    {
        const int m = tid % kTS;
        const int h = __builtin_amdgcn_readfirstlane(tid / kTS);
        float y0 = 0.0f, y1 = 0.0f, y2 = 0.0f;
        if (h < 2) {
            for (int q0 = h * 128; q0 < h * 128 + 128; q0 += 8) {
                const uint4 a8 = *reinterpret_cast<const uint4 *>(&act[m * kStr + q0]);
                const uint32_t w2[4] = {a8.x, a8.y, a8.z, a8.w};
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float x = bf2f((uint16_t)(w2[e / 2] >> (16 * (e % 2))));
                    const int q = q0 + e;
                    y0 += x * Wh[3 * q];
                    y1 += x * Wh[3 * q + 1];
                    y2 += x * Wh[3 * q + 2];
                }
            }
        }
        if (h == 1) {
            yp[0][m] = y0;
            yp[1][m] = y1;
            yp[2][m] = y2;
        }
        __syncthreads();
        if (h == 0) {
            const bool valid = m0 + m < A.B;
            const float y[3] = {y0 + yp[0][m], y1 + yp[1][m], y2 + yp[2][m]};
            double ls = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float dx = P.out_scale * (y[c] + bh[c]);
                const float r = valid ? dx - A.target[c * A.ld + m0 + m] : 0.0f;
                ls += (double)r * (double)r;
                // d loss / d y_c = out_scale * d loss / d dx_c
                const float dy = P.out_scale * (A.mse_scale * r);
                dys[c][m] = dy;
                A.dy[c * A.Bp + m0 + m] = dy;
                if (A.pred && valid) A.pred[c * A.B + m0 + m] = dx;
            }
            lsum[m] = ls;
        }
    }
    __syncthreads();
    // head gradient partials: dW_h[k][c] = sum_m h4[m][k] dy_c[m], db_h[c] = sum_m dy_c[m]
    if (tid < kMlpWidth) {
        const int k = tid;
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
        for (int m = 0; m < kTS; ++m) {
            const float x = bf2f(act[m * kStr + k]);
            s0 += x * dys[0][m];
            s1 += x * dys[1][m];
            s2 += x * dys[2][m];
        }
        float *o = A.part_head + tile * kHeadPart;
        o[3 * k] = s0;
        o[3 * k + 1] = s1;
        o[3 * k + 2] = s2;
        if (k < 3) {
            float b = 0.0f;
            for (int m = 0; m < kTS; ++m) b += dys[k][m];
            o[3 * kMlpWidth + k] = b;
        }
        if (k == 3) {
            double ls = 0.0;
            for (int m = 0; m < kTS; ++m) ls += lsum[m];
            A.part_loss[tile] = ls;
        }
    }
}

__global__ __launch_bounds__(kTT, 4) void train_bwd_kernel(TrainArgs A)
{
    __shared__ __attribute__((aligned(16))) uint16_t act[kTS * kStr];
    __shared__ float dys[3][kTS];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const long long tile = blockIdx.x;
    const long long m0 = tile * kTS;
    const MlpDev &P = A.P;
    if (tid < kTS) {
#pragma unroll
        for (int c = 0; c < 3; ++c) dys[c][tid] = A.dy[c * A.Bp + m0 + tid];
    }
    __syncthreads();
    // dz_3 = (dy W_h^T) * gelu'(z_3), in the accumulator positions of a product
    const float *Wh = P.params + kOffWh;
    const int top = kMlpHidden - 1;
#pragma unroll
    for (int j = 0; j < kNJ; ++j) {
        const int n0 = wave * 16 * kNJ + 16 * j + 4 * (lane / 16);
        float w[4][3];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int c = 0; c < 3; ++c) w[e][c] = Wh[3 * (n0 + e) + c];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int m = 16 * i + lane % 16;
            float d[4], g[4];
            load_frag4(A.dgelu[top] + frag_off(tile, wave, j, i, lane), d);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                g[e] = (dys[0][m] * w[e][0] + dys[1][m] * w[e][1] + dys[2][m] * w[e][2]) * d[e];
            *reinterpret_cast<uint2 *>(&act[m * kStr + n0]) = pack4(g[0], g[1], g[2], g[3]);
        }
    }
    __syncthreads();
    store_t8<kMlpWidth>(act, A.dzt[top], tile, tid);
    for (int l = top; l >= 1; --l) {
        // dh_l = dz_l W_l^T: out^T[k][m] = sum_n W_l[k][n] dz_l[m][n], W_l rows as stored ([in][out])
        f32x4 acc[8][kNJ];
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < kNJ; ++j) acc[i][j] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
        tile_product<kMlpWidth, true>(P.wbf + mlp_off_bf16(l), act, acc, wave, lane);
        __syncthreads();
        const uint16_t *dl = A.dgelu[l - 1];
#pragma unroll
        for (int j = 0; j < kNJ; ++j) {
            const int n0 = wave * 16 * kNJ + 16 * j + 4 * (lane / 16);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                float d[4];
                load_frag4(dl + frag_off(tile, wave, j, i, lane), d);
                *reinterpret_cast<uint2 *>(&act[(16 * i + lane % 16) * kStr + n0]) =
                    pack4(acc[i][j][0] * d[0], acc[i][j][1] * d[1], acc[i][j][2] * d[2],
                          acc[i][j][3] * d[3]);
            }
        }
        __syncthreads();
        store_t8<kMlpWidth>(act, A.dzt[l - 1], tile, tid);
    }
}

// Sum of a fragment's eight BF16 values, in order
__device__ __forceinline__ float sum8(const bf16x8 &v)
{
    const uint4 u = __builtin_bit_cast(uint4, v);
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
    float s = 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        s += __uint_as_float(w[e] << 16);
        s += __uint_as_float(w[e] & 0xffff0000u);
    }
    return s;
}

// Gradient partials of chunk c (rows c*2048 .. +2047), part[c][i] in the
// parameter layout:
//  * hidden weights: part[c][off_w(l) + k*256 + n] = sum over the chunk's rows m
//    of h_l[m][k] dz_l[m][n].  Block = one 128 x 128 output tile of one layer
//    (layer 0: 128 x 256 -> 2 tiles, the others 4) and one chunk; four waves
//    as 2 x 2 of 64 x 64; fragments come straight from the T8 arrays.
//  * hidden biases: part[c][off_b(l) + n] = sum over the rows of dz_l[m][n], by
//    the waves whose tile starts at k = 0, from the dz fragments they load
//    (per lane in row order, then the four lane groups in a fixed order).
//  * head: part[c][off_h + p] = sum of the per-tile head partials of the
//    chunk's tiles in tile order (the last block of each chunk).
__global__ __launch_bounds__(256) void train_wgrad_kernel(TrainArgs A)
{
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    // one-dimensional grid of (tile, chunk) pairs, tile fastest, remapped so
    // that each XCD runs a contiguous run of them: the tiles of one chunk, which
    // read the same activations and gradients, then share that XCD's L2
    const int lin = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    int t = lin % (kWgradTiles + 1);
    const int chunk = lin / (kWgradTiles + 1);
    const long long mb = (long long)chunk * kWgradChunk;
    const long long me = min(mb + kWgradChunk, A.Bp);
    if (t == kWgradTiles) {
        const long long t0 = mb / kTS, t1 = me / kTS;
        for (int p = threadIdx.x; p < kHeadPart; p += 256) {
            float s = 0.0f;
            for (long long q = t0; q < t1; ++q) s += A.part_head[q * kHeadPart + p];
            A.part_w[(long long)chunk * kMlpParams + kOffWh + p] = s;
        }
        return;
    }
    const int l = t < 2 ? 0 : 1 + (t - 2) / 4;
    if (l > 0) t = (t - 2) % 4;
    const int K = mlp_in_width(l);
    const int k0 = (t / 2) * 128 + (wave / 2) * 64, n0 = (t % 2) * 128 + (wave % 2) * 64;
    const bool bias_wave = (k0 == 0);      // wave-uniform
    const uint16_t *H = A.ht[l];
    const uint16_t *D = A.dzt[l];
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
    float bsum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    auto load = [&](long long m, bf16x8 *a, bf16x8 *b) {
        const long long g = m / 8 + lane / 16;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a[i] = *reinterpret_cast<const bf16x8 *>(H + (g * K + k0 + 16 * i + lane % 16) * 8);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            b[j] = *reinterpret_cast<const bf16x8 *>(D + (g * kMlpWidth + n0 + 16 * j + lane % 16) * 8);
    };
    auto step = [&](const bf16x8 *a, const bf16x8 *b) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        if (bias_wave) {
#pragma unroll
            for (int j = 0; j < 4; ++j) bsum[j] += sum8(b[j]);
        }
    };
    bf16x8 a0[4], b0[4], a1[4], b1[4];
    load(mb, a0, b0);
    for (long long m = mb; m < me; m += 64) {
        // rows come in whole tiles of 128, so a chunk holds a multiple of 64 rows
        load(m + 32, a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        step(a0, b0);
        if (m + 64 < me) load(m + 64, a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        step(a1, b1);
    }
    float *out = A.part_w + (long long)chunk * kMlpParams;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + 16 * j + lane % 16;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = k0 + 16 * i + 4 * (lane / 16) + e;
                out[mlp_off_w(l) + (long long)k * kMlpWidth + n] = acc[i][j][e];
            }
        }
    if (bias_wave) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // lane groups g = lane / 16 hold rows 8g .. 8g+7 of every 32: (g0 + g1) + (g2 + g3)
            float v = bsum[j] + __shfl_xor(bsum[j], 16);
            v = v + __shfl_xor(v, 32);
            if (lane < 16) out[mlp_off_b(l) + n0 + 16 * j + lane] = v;
        }
    }
}

// Gradient of every parameter (the chunk partials summed in chunk order), Adam,
// and the BF16 copies; block 0 also sums the per-tile losses (fixed tree).
__global__ __launch_bounds__(256) void train_update_kernel(TrainArgs A, AdamArgs ad)
{
    __shared__ double ls[256];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < kMlpParams) {
        // the partials in chunk order, eight loads in flight before their adds
        float g = 0.0f;
        int c = 0;
        for (; c + 8 <= A.n_chunks; c += 8) {
            float p[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) p[e] = A.part_w[(long long)(c + e) * kMlpParams + i];
#pragma unroll
            for (int e = 0; e < 8; ++e) g += p[e];
        }
        for (; c < A.n_chunks; ++c) g += A.part_w[(long long)c * kMlpParams + i];
        if (A.grads) A.grads[i] = g;
        const float mi = ad.beta1 * A.m[i] + (1.0f - ad.beta1) * g;
        const float vi = ad.beta2 * A.v[i] + (1.0f - ad.beta2) * g * g;
        A.m[i] = mi;
        A.v[i] = vi;
        const float pi = A.params[i] - ad.lr * (mi * ad.c1) / (sqrtf(vi * ad.c2) + ad.eps);
        A.params[i] = pi;
        // BF16 copies of the hidden weights, [in][out] and [out][in], in fragment order
        int l = 0;
        while (l + 1 < kMlpHidden && i >= mlp_off_w(l + 1)) ++l;
        if (i < kOffWh && i < mlp_off_b(l)) {
            const long long r = i - mlp_off_w(l);
            const int K = mlp_in_width(l);
            const int k = (int)(r / kMlpWidth), n = (int)(r % kMlpWidth);
            const uint16_t b = __builtin_bit_cast(uint16_t, (__bf16)pi);
            A.wbf[mlp_off_bf16(l) + frag_index(k, n, kMlpWidth)] = b;
            A.wbf[mlp_off_bf16(l) + (long long)K * kMlpWidth + frag_index(n, k, K)] = b;
        }
    }
    if (blockIdx.x == 0 && A.loss) {
        double v = 0.0;
        for (long long c = threadIdx.x; c < A.n_tiles; c += 256) v += A.part_loss[c];
        ls[threadIdx.x] = v;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) ls[threadIdx.x] += ls[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) *A.loss = ls[0] * A.loss_mult;
    }
}

}  // namespace

hipError_t launch_train_step(const TrainArgs &a, const AdamArgs &ad, hipStream_t s)
{
    const unsigned nt = (unsigned)a.n_tiles;
    {
        LaunchTimer timer("train_fwd_kernel", s);
        hipLaunchKernelGGL(train_fwd_kernel, dim3(nt), dim3(kTT), 0, s, a);
        timer.stop(s);
    }
    {
        LaunchTimer timer("train_bwd_kernel", s);
        hipLaunchKernelGGL(train_bwd_kernel, dim3(nt), dim3(kTT), 0, s, a);
        timer.stop(s);
    }
    {
        LaunchTimer timer("train_wgrad_kernel", s);
        hipLaunchKernelGGL(train_wgrad_kernel, dim3((unsigned)((kWgradTiles + 1) * a.n_chunks)),
                           dim3(256), 0, s, a);
        timer.stop(s);
    }
    {
        LaunchTimer timer("train_update_kernel", s);
        hipLaunchKernelGGL(train_update_kernel, dim3((unsigned)((kMlpParams + 255) / 256)), dim3(256), 0,
                           s, a, ad);
        timer.stop(s);
    }
    return hipGetLastError();
}

}  // namespace lcs
