// mlp.hip -- Fourier-feature MLP flow-map surrogate on gfx950: features,
// BF16 MFMA layers with FP32 accumulation, head, loss gradient, backward and
// Adam.  The surrogate approximates the flow map over a window tau locally in
// space and time (the paper's discussion cites local flow-map approximation
// as a way to save interpolation work when flow maps are wanted for many
// start times, Sec. 4); plain RK4 stays the fallback and the reference.
//
// Matrix products use v_mfma_f32_16x16x32_bf16 (16x16 output tile, K = 32 per
// instruction).  Lane layout (checked on the device): A fragment = row l%16,
// k = 8*(l/16) .. +7; B fragment = column l%16, same k; D = rows
// 4*(l/16) .. +3 of column l%16.

#include "lcs_internal.h"

namespace lcs {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// tanh form of GELU and its derivative (FP32)
__device__ __forceinline__ float gelu(float z)
{
    const float c = 0.7978845608028654f;
    return 0.5f * z * (1.0f + tanhf(c * (z + 0.044715f * z * z * z)));
}

__device__ __forceinline__ float gelu_prime(float z)
{
    const float c = 0.7978845608028654f;
    const float t = tanhf(c * (z + 0.044715f * z * z * z));
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * c * (1.0f + 3.0f * 0.044715f * z * z);
}

// ---------------------------------------------------------------------------
// Fourier features: H0[m][f] = cos(2 pi B_f . v), H0[m][64+f] = sin(...)
// ---------------------------------------------------------------------------
// one thread per (sample m, frequency f), f fastest, so that the BF16 stores of
// a wave fill consecutive bytes of the sample rows
__global__ __launch_bounds__(256) void features_kernel(MlpDev P, const float *__restrict__ xt,
                                                       long long M, uint16_t *__restrict__ H0)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * kMlpFreq) return;
    const long long m = idx / kMlpFreq;
    const int f = (int)(idx - m * kMlpFreq);
    float v[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) v[a] = (xt[a * M + m] - P.in_shift[a]) * P.in_scale[a];
    uint16_t *row = H0 + m * kMlpFeat;
    const float *b = P.freq + 4 * f;
    const float ph = b[0] * v[0] + b[1] * v[1] + b[2] * v[2] + b[3] * v[3];
    float s, c;
    sincospif(2.0f * ph, &s, &c);
    row[f] = f2bf(c);
    row[kMlpFreq + f] = f2bf(s);
}

// ---------------------------------------------------------------------------
// C[M][N] = A[M][K] * Bt[N][K]^T in BF16 with FP32 accumulation.
// Block tile 128 x 128, k-step 32, four waves as 2 x 2 of 64 x 64 (4 x 4 MFMA
// tiles each).  EPI_FWD: z = C + bias -> Z (optional) and H = gelu(z), both
// BF16.  EPI_BWD: dZ = C * gelu'(Zprev), BF16.
// ---------------------------------------------------------------------------
constexpr int EPI_FWD = 0;
constexpr int EPI_BWD = 1;
constexpr int kBM = 128, kBN = 128, kBK = 32, kLdsStride = kBK + 8;

template <int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kBM * kLdsStride];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN * kLdsStride];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wm = wave / 2, wn = wave % 2;
    const long long m0 = (long long)blockIdx.y * kBM;
    const int n0 = blockIdx.x * kBN;
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};

    for (int k0 = 0; k0 < g.K; k0 += kBK) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int c = tid + 256 * r;          // 512 chunks of 8 BF16 per tile
            const int row = c / 4, kc = (c % 4) * 8;
            uint4 va = make_uint4(0, 0, 0, 0);
            if (m0 + row < g.M)
                va = *reinterpret_cast<const uint4 *>(g.A + (m0 + row) * g.K + k0 + kc);
            *reinterpret_cast<uint4 *>(&As[row * kLdsStride + kc]) = va;
            const long long bo = g.bt_frag ? frag_index(n0 + row, k0 + kc, g.K)
                                           : (long long)(n0 + row) * g.K + k0 + kc;
            const uint4 vb = *reinterpret_cast<const uint4 *>(g.Bt + bo);
            *reinterpret_cast<uint4 *>(&Bs[row * kLdsStride + kc]) = vb;
        }
        __syncthreads();
        bf16x8 af[4], bfr[4];
        const int ko = 8 * (lane / 16);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = wm * 64 + 16 * i + lane % 16;
            af[i] = *reinterpret_cast<const bf16x8 *>(&As[row * kLdsStride + ko]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = wn * 64 + 16 * j + lane % 16;
            bfr[j] = *reinterpret_cast<const bf16x8 *>(&Bs[col * kLdsStride + ko]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + wn * 64 + 16 * j + lane % 16;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const long long m = m0 + wm * 64 + 16 * i + 4 * (lane / 16) + e;
                if (m >= g.M) continue;
                const long long o = m * g.N + n;
                if constexpr (EPI == EPI_FWD) {
                    const float z = acc[i][j][e] + g.bias[n];
                    if (g.Z) g.Z[o] = f2bf(z);
                    g.H[o] = f2bf(gelu(z));
                } else {
                    g.H[o] = f2bf(acc[i][j][e] * gelu_prime(bf2f(g.Z[o])));
                }
            }
        }
}

// ---------------------------------------------------------------------------
// Weight gradient: part[chunk][K][N] = sum over the chunk's rows m of
// X[m][k] * D[m][n].  Block tile 64 x 64, m-step 32, four waves as 2 x 2 of
// 32 x 32.  Tiles are stored transposed in LDS ([k][m], [n][m]) so that the
// MFMA fragments read contiguous m.
// ---------------------------------------------------------------------------
constexpr int kWT = 64, kWStep = 32, kWStride = kWStep + 8;

__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t Xs[kWT * kWStride];
    __shared__ __attribute__((aligned(16))) uint16_t Ds[kWT * kWStride];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const int wk = wave / 2, wn = wave % 2;
    const int k0 = blockIdx.y * kWT, n0 = blockIdx.x * kWT;
    const long long mb = (long long)blockIdx.z * g.chunk;
    const long long me = min(mb + g.chunk, g.M);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.0f, 0.0f, 0.0f, 0.0f};
    const int mm = tid / 8, cc = (tid % 8) * 8;   // 32 rows x 8 chunks of 8 values
    for (long long m = mb; m < me; m += kWStep) {
        uint4 vx = make_uint4(0, 0, 0, 0), vd = make_uint4(0, 0, 0, 0);
        if (m + mm < me) {
            vx = *reinterpret_cast<const uint4 *>(g.X + (m + mm) * g.K + k0 + cc);
            vd = *reinterpret_cast<const uint4 *>(g.D + (m + mm) * g.N + n0 + cc);
        }
        const uint16_t *px = reinterpret_cast<const uint16_t *>(&vx);
        const uint16_t *pd = reinterpret_cast<const uint16_t *>(&vd);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            Xs[(cc + e) * kWStride + mm] = px[e];
            Ds[(cc + e) * kWStride + mm] = pd[e];
        }
        __syncthreads();
        const int ko = 8 * (lane / 16);
        bf16x8 af[2], bfr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            af[i] = *reinterpret_cast<const bf16x8 *>(&Xs[(wk * 32 + 16 * i + lane % 16) * kWStride + ko]);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            bfr[j] = *reinterpret_cast<const bf16x8 *>(&Ds[(wn * 32 + 16 * j + lane % 16) * kWStride + ko]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    float *out = g.part + (long long)blockIdx.z * g.K * g.N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn * 32 + 16 * j + lane % 16;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = k0 + wk * 32 + 16 * i + 4 * (lane / 16) + e;
                out[(long long)k * g.N + n] = acc[i][j][e];
            }
        }
}

// Column sums of D over each chunk: part[chunk][n] = sum_m D[m][n] (bias grads).
__global__ __launch_bounds__(256) void colsum_kernel(const uint16_t *__restrict__ D, long long M,
                                                     int N, long long chunk, float *__restrict__ part)
{
    const int n = threadIdx.x;
    const long long mb = (long long)blockIdx.x * chunk;
    const long long me = min(mb + chunk, M);
    float s = 0.0f;
    if (n < N)
        for (long long m = mb; m < me; ++m) s += bf2f(D[m * N + n]);
    if (n < N) part[(long long)blockIdx.x * N + n] = s;
}

// out[i] = sum over c < nchunk of part[c*len + i] (fixed order: deterministic).
__global__ __launch_bounds__(256) void reduce_chunks_kernel(const float *__restrict__ part, int nchunk,
                                                            long long len, float *__restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += part[(long long)c * len + i];
    out[i] = s;
}

// The same sum for short outputs with many chunks (bias and head gradients):
// a block takes 64 consecutive outputs and four chunk groups; thread (g, o)
// sums chunks g, g + 4, g + 8, ... of output o in order (a wave reads 64
// adjacent floats of one chunk per load), then the four group sums are added
// in group order (deterministic).
__global__ __launch_bounds__(256) void reduce_chunks_tree_kernel(const float *__restrict__ part,
                                                                 int nchunk, long long len,
                                                                 float *__restrict__ out)
{
    __shared__ float sh[4][64];
    const int o = threadIdx.x % 64, grp = threadIdx.x / 64;
    const long long i = (long long)blockIdx.x * 64 + o;
    float s = 0.0f;
    if (i < len)
        for (int c = grp; c < nchunk; c += 4) s += part[(long long)c * len + i];
    sh[grp][o] = s;
    __syncthreads();
    if (grp == 0 && i < len) out[i] = ((sh[0][o] + sh[1][o]) + sh[2][o]) + sh[3][o];
}

// ---------------------------------------------------------------------------
// Head: dx[c][m] = out_scale * (sum_k H4[m][k] Wh[k][c] + bh[c]), FP32.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void head_fwd_kernel(MlpDev P, const uint16_t *__restrict__ H4,
                                                       long long M, float *__restrict__ dx)
{
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const float *Wh = P.params + kOffWh;
    const float *bh = P.params + kOffBh;
    float y0 = 0.0f, y1 = 0.0f, y2 = 0.0f;
    const uint4 *row = reinterpret_cast<const uint4 *>(H4 + m * kMlpWidth);
    for (int q = 0; q < kMlpWidth / 8; ++q) {
        const uint4 v = row[q];
        const uint16_t *h = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 8 * q + e;
            const float x = bf2f(h[e]);
            y0 += x * Wh[3 * k];
            y1 += x * Wh[3 * k + 1];
            y2 += x * Wh[3 * k + 2];
        }
    }
    dx[m] = P.out_scale * (y0 + bh[0]);
    dx[M + m] = P.out_scale * (y1 + bh[1]);
    dx[2 * M + m] = P.out_scale * (y2 + bh[2]);
}

// Head backward, per (m, k): dy = out_scale * ddx[:, m];
// dZ4[m][k] = (sum_c dy_c Wh[k][c]) * gelu'(Z4[m][k]).
__global__ __launch_bounds__(256) void head_bwd_data_kernel(MlpDev P, const float *__restrict__ ddx,
                                                            const uint16_t *__restrict__ Z4, long long M,
                                                            uint16_t *__restrict__ dZ4)
{
    const long long m = blockIdx.x;
    const int k = threadIdx.x;
    const float *Wh = P.params + kOffWh;
    const float d0 = P.out_scale * ddx[m], d1 = P.out_scale * ddx[M + m],
                d2 = P.out_scale * ddx[2 * M + m];
    const float dh = d0 * Wh[3 * k] + d1 * Wh[3 * k + 1] + d2 * Wh[3 * k + 2];
    const long long o = m * kMlpWidth + k;
    dZ4[o] = f2bf(dh * gelu_prime(bf2f(Z4[o])));
}

// Head weight/bias partial gradients over a chunk of rows:
// part[chunk][k*3 + c] = sum_m H4[m][k] dy_c[m]; part[chunk][768 + c] = sum_m dy_c[m].
__global__ __launch_bounds__(256) void head_wgrad_kernel(MlpDev P, const float *__restrict__ ddx,
                                                         const uint16_t *__restrict__ H4, long long M,
                                                         long long chunk, float *__restrict__ part)
{
    const int k = threadIdx.x;
    const long long mb = (long long)blockIdx.x * chunk;
    const long long me = min(mb + chunk, M);
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, b0 = 0.0f, b1 = 0.0f, b2 = 0.0f;
    for (long long m = mb; m < me; ++m) {
        const float d0 = P.out_scale * ddx[m], d1 = P.out_scale * ddx[M + m],
                    d2 = P.out_scale * ddx[2 * M + m];
        const float h = bf2f(H4[m * kMlpWidth + k]);
        s0 += h * d0;
        s1 += h * d1;
        s2 += h * d2;
        b0 += d0;
        b1 += d1;
        b2 += d2;
    }
    float *o = part + (long long)blockIdx.x * kHeadPart;
    o[3 * k] = s0;
    o[3 * k + 1] = s1;
    o[3 * k + 2] = s2;
    if (k == 0) {
        o[3 * kMlpWidth] = b0;
        o[3 * kMlpWidth + 1] = b1;
        o[3 * kMlpWidth + 2] = b2;
    }
}

// ---------------------------------------------------------------------------
// Loss gradient, Adam, BF16 weight copies
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mse_grad_kernel(const float *__restrict__ pred,
                                                       const float *__restrict__ target, long long n,
                                                       float scale, float *__restrict__ grad)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) grad[i] = scale * (pred[i] - target[i]);
}

// Sum of squared errors in one workgroup, fixed order (deterministic).
__global__ __launch_bounds__(1024) void sse_kernel(const float *__restrict__ pred,
                                                   const float *__restrict__ target, long long n,
                                                   double *__restrict__ out, double mult)
{
    __shared__ double red[1024];
    double s = 0.0;
    for (long long i = threadIdx.x; i < n; i += 1024) {
        const double d = (double)pred[i] - (double)target[i];
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * mult;
}

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p, const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   long long n, AdamArgs a)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = a.beta1 * m[i] + (1.0f - a.beta1) * gi;
    const float vi = a.beta2 * v[i] + (1.0f - a.beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mhat = mi * a.c1, vhat = vi * a.c2;
    p[i] = p[i] - a.lr * mhat / (sqrtf(vhat) + a.eps);
}

// BF16 copies of the four hidden-layer matrices, both in fragment order
// (frag_index): W_l ([K][N], as stored) and W_l^T ([N][K]).
__global__ __launch_bounds__(256) void refresh_bf16_kernel(const float *__restrict__ params,
                                                           uint16_t *__restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kBf16Count / 2) return;
    // locate layer l and element (k, n) of its [K][N] matrix
    int l = 0;
    long long r = i;
    while (r >= (long long)mlp_in_width(l) * kMlpWidth) {
        r -= (long long)mlp_in_width(l) * kMlpWidth;
        ++l;
    }
    const int K = mlp_in_width(l);
    const int k = (int)(r / kMlpWidth), n = (int)(r % kMlpWidth);
    const uint16_t b = f2bf(params[mlp_off_w(l) + r]);
    out[mlp_off_bf16(l) + frag_index(k, n, kMlpWidth)] = b;         // W, fragment order
    out[mlp_off_bf16(l) + (long long)K * kMlpWidth + frag_index(n, k, K)] = b;   // W^T, fragment order
}

// ---------------------------------------------------------------------------
// Fused surrogate composition: a workgroup owns 128 consecutive seeds and runs
// every window for them -- features, the four hidden layers on MFMA and the
// head -- with the activations resident in LDS; weights stream from L2 as
// MFMA B fragments.  x_{k+1} = x_k + dx(x_k, t0 + k tau).
// ---------------------------------------------------------------------------
constexpr int kFT = 128;                  // samples per workgroup
constexpr int kActStride = kMlpWidth + 8; // BF16 per LDS row (16-byte aligned rows)

// tanh-form GELU written as z * sigmoid(2u) = z / (1 + exp(-2u)) with
// u = sqrt(2/pi) (z + 0.044715 z^3), and -2u log2(e) folded into
// z (A + B z^2): one multiply, one FMA and one multiply before the base-2
// exponential, then the hardware reciprocal (the result is rounded to BF16
// next; the folding moves it by at most ~5e-7 absolute)
__device__ __forceinline__ float gelu_fast(float z)
{
    constexpr float A = -2.3022082f;    // -2 log2(e) sqrt(2/pi)
    constexpr float B = -0.10294324f;   // A * 0.044715
    const float w = fmaf(B, z * z, A);
    return z * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z * w));
}

// Four floats rounded to BF16 (to nearest even) and packed in 8 bytes, two
// per conversion.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint2 pack_bf16x4(float a, float b, float c, float d)
{
    const bf16x2 lo = __builtin_convertvector((f32x2){a, b}, bf16x2);
    const bf16x2 hi = __builtin_convertvector((f32x2){c, d}, bf16x2);
    return make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
}

constexpr int kCT = 512;                  // threads per composition workgroup (8 waves)

__global__ __launch_bounds__(kCT, 2) void compose_fused_kernel(ComposeArgs A)
{
    __shared__ __attribute__((aligned(16))) uint16_t act[kFT * kActStride];
    __shared__ float xs[3][kFT];
    __shared__ float yp[3][kFT];
    static_assert(2 * kFT == 256 && kMlpWidth == 256, "the head splits 256 inputs over 2 x 128 threads");
    static_assert(kCT / kWave * 32 == kMlpWidth, "each wave owns 32 output columns");
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const long long s0 = (long long)blockIdx.x * kFT;
    const SeedTiling &g = A.g;
    if (tid < kFT) {
        const long long s = min(s0 + tid, A.ns - 1);
        const long long c[3] = {s % g.sn[0], (s / g.sn[0]) % g.sn[1],
                                s / ((long long)g.sn[0] * g.sn[1])};
#pragma unroll
        for (int a = 0; a < 3; ++a) xs[a][tid] = (float)(g.s_origin[a] + (double)c[a] * g.s_spacing[a]);
    }
    __syncthreads();
    const MlpDev &P = A.P;
    const float *Wh = P.params + kOffWh;
    const float *bh = P.params + kOffBh;
    for (int k = 0; k < A.n_windows; ++k) {
        const float tk = (float)(A.t0 + (double)k * A.tau);
        // features: thread -> (sample m, frequency f), f fastest
        for (int idx = tid; idx < kFT * kMlpFreq; idx += kCT) {
            const int m = idx / kMlpFreq, f = idx % kMlpFreq;
            const float v0 = (xs[0][m] - P.in_shift[0]) * P.in_scale[0];
            const float v1 = (xs[1][m] - P.in_shift[1]) * P.in_scale[1];
            const float v2 = (xs[2][m] - P.in_shift[2]) * P.in_scale[2];
            const float v3 = (tk - P.in_shift[3]) * P.in_scale[3];
            const float *b = P.freq + 4 * f;
            // B_f . v in revolutions, reduced exactly to [-1/2, 1/2], then the
            // hardware sine and cosine of 2 pi r (the features are rounded to
            // BF16, far coarser than their error)
            const float rev = b[0] * v0 + b[1] * v1 + b[2] * v2 + b[3] * v3;
            const float r = rev - rintf(rev);
            act[m * kActStride + f] = f2bf(__builtin_amdgcn_cosf(r));
            act[m * kActStride + kMlpFreq + f] = f2bf(__builtin_amdgcn_sinf(r));
        }
        __syncthreads();
        for (int l = 0; l < kMlpHidden; ++l) {
            const int K = mlp_in_width(l);
            const uint16_t *Wt = P.wbf + mlp_off_bf16(l) + (long long)K * kMlpWidth;   // W^T, fragment order
            const float *bias = P.params + mlp_off_b(l);
            // the transposed product out^T[n][m] = sum_k W^T[n][k] act[m][k]: weights
            // as the A operand, activations as B, so that a lane's four results
            // are four consecutive output columns n of one sample m; wave w owns
            // columns 32w .. 32w+31.  The accumulators start from the bias.
            f32x4 acc[8][2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int n0 = wave * 32 + 16 * j + 4 * (lane / 16);
                const f32x4 b4 = (f32x4){bias[n0], bias[n0 + 1], bias[n0 + 2], bias[n0 + 3]};
#pragma unroll
                for (int i = 0; i < 8; ++i) acc[i][j] = b4;
            }
            const int ko = 8 * (lane / 16);
            // a wave's weight fragment of one 16 x 32 block: 1 KiB contiguous
            auto load_w = [&](int kk, bf16x8 *w) {
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    w[j] = *reinterpret_cast<const bf16x8 *>(
                        Wt + (uint32_t)(((wave * 2 + j) * (K / 32) + kk / 32) * 512 + lane * 8));
            };
            auto mfma_slice = [&](int kk, const bf16x8 *w) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const bf16x8 xfr = *reinterpret_cast<const bf16x8 *>(
                        &act[(16 * i + lane % 16) * kActStride + kk + ko]);
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[j], xfr, acc[i][j], 0, 0, 0);
                }
            };
            // two fragment buffers: the next slice's weights are in flight from L2
            // while the current slice's products run (K is a multiple of 64)
            static_assert(kMlpFeat % 64 == 0 && kMlpWidth % 64 == 0, "K must be a multiple of 64");
            bf16x8 wa[2], wb[2];
            load_w(0, wa);
            for (int kk = 0; kk < K; kk += 64) {
                load_w(kk + 32, wb);
                __builtin_amdgcn_sched_barrier(0);
                mfma_slice(kk, wa);
                if (kk + 64 < K) load_w(kk + 64, wa);
                __builtin_amdgcn_sched_barrier(0);
                mfma_slice(kk + 32, wb);
            }
            __syncthreads();   // every wave has read this layer's input
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int n0 = wave * 32 + 16 * j + 4 * (lane / 16);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int m = 16 * i + lane % 16;
                    *reinterpret_cast<uint2 *>(&act[m * kActStride + n0]) =
                        pack_bf16x4(gelu_fast(acc[i][j][0]), gelu_fast(acc[i][j][1]),
                                    gelu_fast(acc[i][j][2]), gelu_fast(acc[i][j][3]));
                }
            }
            __syncthreads();
        }
        // head: two threads per sample (waves 0-3), each summing half of the 256
        // inputs; the half is uniform over a wave (waves 0-1 the first, 2-3 the
        // second), so the head weights are scalar loads, and the second half's
        // partial sums reach the first through LDS
        {
            const int m = tid % kFT;
            const int h = __builtin_amdgcn_readfirstlane(tid / kFT);
            float y0 = 0.0f, y1 = 0.0f, y2 = 0.0f;
            if (h < 2) {
                for (int q0 = h * 128; q0 < h * 128 + 128; q0 += 8) {
                    // eight activations in one 16-byte LDS read (rows are 16-byte aligned)
                    const uint4 a8 = *reinterpret_cast<const uint4 *>(&act[m * kActStride + q0]);
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
            __syncthreads();   // all head reads of act done before the next window's features
            if (h == 0) {
                xs[0][m] += P.out_scale * ((y0 + yp[0][m]) + bh[0]);
                xs[1][m] += P.out_scale * ((y1 + yp[1][m]) + bh[1]);
                xs[2][m] += P.out_scale * ((y2 + yp[2][m]) + bh[2]);
            }
            __syncthreads();
        }
    }
    if (tid < kFT && s0 + tid < A.ns) {
#pragma unroll
        for (int a = 0; a < 3; ++a) A.xf[a * A.ns + s0 + tid] = xs[a][tid];
    }
}

__global__ __launch_bounds__(256) void sub_kernel(const float *__restrict__ a, const float *__restrict__ b,
                                                  long long n, float *__restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] - b[i];
}

}  // namespace

hipError_t launch_compose_fused(const ComposeArgs &a, hipStream_t s)
{
    LaunchTimer timer("compose_fused_kernel", s);
    hipLaunchKernelGGL(compose_fused_kernel, dim3((unsigned)((a.ns + kFT - 1) / kFT)), dim3(kCT), 0, s, a);
    timer.stop(s);
    return hipGetLastError();
}

hipError_t launch_sub(const float *a, const float *b, long long n, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(sub_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_features(const MlpDev &P, const float *xt, long long M, uint16_t *H0, hipStream_t s)
{
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((M * kMlpFreq + 255) / 256)), dim3(256), 0, s,
                       P, xt, M, H0);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs &g, bool backward, hipStream_t s)
{
    dim3 grid((unsigned)(g.N / kBN), (unsigned)((g.M + kBM - 1) / kBM)), block(256);
    LaunchTimer timer(backward ? "gemm_kernel<EPI_BWD>" : "gemm_kernel<EPI_FWD>", s);
    if (backward) hipLaunchKernelGGL(gemm_kernel<EPI_BWD>, grid, block, 0, s, g);
    else hipLaunchKernelGGL(gemm_kernel<EPI_FWD>, grid, block, 0, s, g);
    timer.stop(s);
    return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs &g, int nchunk, hipStream_t s)
{
    dim3 grid((unsigned)(g.N / kWT), (unsigned)(g.K / kWT), (unsigned)nchunk), block(256);
    LaunchTimer timer("wgrad_kernel", s);
    hipLaunchKernelGGL(wgrad_kernel, grid, block, 0, s, g);
    timer.stop(s);
    return hipGetLastError();
}

hipError_t launch_colsum(const uint16_t *D, long long M, int N, long long chunk, int nchunk,
                         float *part, hipStream_t s)
{
    hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)nchunk), dim3(256), 0, s, D, M, N, chunk, part);
    return hipGetLastError();
}

hipError_t launch_reduce_chunks(const float *part, int nchunk, long long len, float *out, hipStream_t s)
{
    if (len <= 0) return hipSuccess;
    if (len <= 4096 && nchunk > 64)
        hipLaunchKernelGGL(reduce_chunks_tree_kernel, dim3((unsigned)((len + 63) / 64)), dim3(256), 0, s,
                           part, nchunk, len, out);
    else
        hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s,
                           part, nchunk, len, out);
    return hipGetLastError();
}

hipError_t launch_head_fwd(const MlpDev &P, const uint16_t *H4, long long M, float *dx, hipStream_t s)
{
    hipLaunchKernelGGL(head_fwd_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, P, H4,
                       M, dx);
    return hipGetLastError();
}

hipError_t launch_head_bwd(const MlpDev &P, const float *ddx, const uint16_t *Z4, const uint16_t *H4,
                           long long M, uint16_t *dZ4, long long chunk, int nchunk, float *part,
                           hipStream_t s)
{
    hipLaunchKernelGGL(head_bwd_data_kernel, dim3((unsigned)M), dim3(kMlpWidth), 0, s, P, ddx, Z4, M,
                       dZ4);
    hipLaunchKernelGGL(head_wgrad_kernel, dim3((unsigned)nchunk), dim3(kMlpWidth), 0, s, P, ddx, H4,
                       M, chunk, part);
    return hipGetLastError();
}

hipError_t launch_mse(const float *pred, const float *target, long long n, float scale, float *grad,
                      double *loss, double loss_mult, hipStream_t s)
{
    if (grad)
        hipLaunchKernelGGL(mse_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pred,
                           target, n, scale, grad);
    if (loss) hipLaunchKernelGGL(sse_kernel, dim3(1), dim3(1024), 0, s, pred, target, n, loss, loss_mult);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, long long n, const AdamArgs &a,
                       hipStream_t s)
{
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, a);
    return hipGetLastError();
}

hipError_t launch_refresh_bf16(const float *params, uint16_t *out, hipStream_t s)
{
    const long long n = kBf16Count / 2;
    hipLaunchKernelGGL(refresh_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params,
                       out);
    return hipGetLastError();
}

}  // namespace lcs
