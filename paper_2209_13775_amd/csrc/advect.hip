// advect.hip -- RK4 flow-map kernels for gfx950.
//
// One lane = one tracer.  The whole integration (all N steps, all four RK4
// stages) runs inside one kernel with the tracer state in registers; the
// paper split every stage into its own kernel to fit Kepler's 31-register
// budget (Sec. 3.1), which CDNA's 512-VGPR lanes do not need.
//
// Per evaluation (Sec. 2 Interpolator; Sec. 3.2): locate the cell on each
// axis, take the 2^D corners of the two frames that bracket t (from the
// tracer's register cache of the cell it sampled last, else gathered from the
// frames in their layout), multilinear weights in space, then linear in time.
// Seeds and positions are carried as two-floats (hi + lo) and the stage
// points as two-float grid-index coordinates: chaotic flows amplify any start
// or position rounding by exp(sigma T), so only the FP32 interpolation
// arithmetic itself is left to round.

#include <stdio.h>

#include "lcs_internal.h"
#include "device_common.h"

// Occupancy of the RK4 advection kernels: at least LCS_RK4_MIN_WAVES waves per
// SIMD (4: at most 128 VGPRs), measured faster than the larger register budget
// the compiler picks by itself; the Adams-Bashforth kernels keep the
// compiler's budget (capped, they spill and slow down).
#ifndef LCS_RK4_MIN_WAVES
#define LCS_RK4_MIN_WAVES 4
#endif
#define LCS_RK4_BOUNDS __launch_bounds__(256, LCS_RK4_MIN_WAVES)
#define LCS_AB_BOUNDS __launch_bounds__(256)

namespace lcs {
namespace {

constexpr uint32_t kOut = LCS_FLAG_OUT;
constexpr uint32_t kNonFinite = LCS_FLAG_NONFINITE;
constexpr uint32_t kTimeOut = LCS_FLAG_TIME_OUT;

// Grid-index coordinate s = (x - origin)/h of the two-float point xh + xl
// along one axis, as a two-float: the difference and the product are formed in
// two-float arithmetic (the product's rounding error recovered with an FMA),
// so s is accurate to FP32 rounding of its fraction rather than of the
// unwrapped position.
__device__ __forceinline__ void to_index(const VelDev &v, int a, float xh, float xl, float &sh,
                                         float &sl)
{
    float dh, dl;
    two_sum(xh, -v.oh[a], dh, dl);
    dl += xl - v.ol[a];
    sh = dh * v.ih[a];
    sl = fmaf(dh, v.ih[a], -sh) + fmaf(dh, v.il[a], dl * v.ih[a]);
}

// Lower node, upper node and local coordinate of the grid-index point
// sh + sl along one axis.  Non-periodic: node = floor(s) limited to [0, n-2].
// Periodic: s folded into [0, n) by whole periods (exact); a fold landing on
// n is node 0.  s is clamped before any float->int conversion, so every input
// (NaN included) yields in-range node indices.
__device__ __forceinline__ void locate_s(const VelDev &v, int a, float sh, float sl, int &lo,
                                         int &hi, float &xi)
{
    const int n = v.n[a];
    const float nf = v.nf[a];
    if ((v.periodic_mask >> a) & 1u) {
        float f = sh - nf * floorf(sh * (1.0f / nf));   // exact: sh minus a multiple of n
        f = fminf(fmaxf(f, 0.0f), nf);
        int i = (int)f;
        float fr = (f - (float)i) + sl;
        if (i >= n) { i = 0; fr = sl; }
        lo = i;
        hi = (i + 1 == n) ? 0 : i + 1;
        xi = fr;
    } else {
        const float f = fminf(fmaxf(sh, 0.0f), nf - 1.0f);
        const int i = min((int)f, n - 2);
        lo = i;
        hi = i + 1;
        xi = (sh - (float)i) + sl;
    }
}

// Frame pair bracketing t and the time weight (FP64 in, FP32 weight out).  t
// is the same for every lane of a wave in the grid kernels, so the frame
// index is made explicitly wave-uniform (it then addresses through SGPRs).
__device__ __forceinline__ void frame_at(const VelDev &v, double t, long long &base, float &alpha)
{
    double tau = (t - v.t_first) * v.inv_dt_frame;
    tau = fmin(fmax(tau, 0.0), (double)(v.n_frames - 1));
    int f = min((int)floor(tau), v.n_frames - 2);
    alpha = (float)(tau - (double)f);
    base = (long long)f * v.frame_stride;
}

__device__ __forceinline__ void frame_at_uniform(const VelDev &v, double t, long long &base,
                                                 float &alpha)
{
    double tau = (t - v.t_first) * v.inv_dt_frame;
    tau = fmin(fmax(tau, 0.0), (double)(v.n_frames - 1));
    const int f = __builtin_amdgcn_readfirstlane(min((int)floor(tau), v.n_frames - 2));
    alpha = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint((float)(tau - (double)f))));
    base = (long long)f * v.frame_stride;
}

// Frame layouts: structure of arrays (one array per component; the x pair
// (i, i+1) of a cell row is one 8-byte load per component), interleaved
// records (2, 3 or 4 floats per node with the components together; one 12-byte
// load per node in 3D, one 16-byte load per x pair in 2D) or time-paired
// records (both frames of a pair per node, 2*dim floats, an extra node per x
// row; the x pair of a cell row in both frames is three 16-byte loads in 3D,
// two in 2D).  Every load
// is a 32-bit byte offset from a wave-uniform frame base.

// Corner values of the cell a tracer sampled last, for both frames of the
// pair, kept in registers: consecutive RK4 stage points mostly fall in the
// same cell of the same frame pair (frames change only every dt_frame/dt
// steps), and then the gathers are skipped.  The values are the same either
// way, so the result does not depend on whether the cache is used.
#ifndef LCS_CELL_CACHE
#define LCS_CELL_CACHE 1
#endif

template <int D>
struct CellCache {
    static constexpr int R = (D == 2) ? 2 : 4;    // rows of 2 corners
    uint32_t node = ~0u;      // byte offset of the cached cell's lower corner (~0u: empty)
    long long base = -1;      // frame base of the cached pair
    float c[2][R][2][D];      // [frame f/f+1][row][lower/upper node][component]
};

// Bytes at a 32-bit offset from a (wave-uniform) frame base.
template <typename T>
__device__ __forceinline__ T load_at(const char *base, uint32_t off)
{
    T v;
    __builtin_memcpy(&v, base + off, sizeof(T));
    return v;
}

// Structure of arrays: one 8-byte pair load per (row, frame, component).
template <int D>
__device__ __forceinline__ void gather_cell_soa(const VelDev &v, long long base,
                                                const uint32_t *rowb, uint32_t pxb, bool wrap,
                                                float (&c)[2][CellCache<D>::R][2][D])
{
    constexpr int R = CellCache<D>::R;
    const long long fs = v.frame_stride;
    float2 pa[D][R], pb[D][R];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const char *__restrict__ A = reinterpret_cast<const char *>(v.u[k] + base);
        const char *__restrict__ B = reinterpret_cast<const char *>(v.u[k] + base + fs);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            pa[k][r] = load_at<float2>(A, rowb[r] + pxb);
            pb[k][r] = load_at<float2>(B, rowb[r] + pxb);
        }
    }
    if (wrap) {
        // cell (n0-1, 0): the loaded pair is (n0-2, n0-1); shift it and fetch node 0
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const char *__restrict__ A = reinterpret_cast<const char *>(v.u[k] + base);
            const char *__restrict__ B = reinterpret_cast<const char *>(v.u[k] + base + fs);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                pa[k][r] = make_float2(pa[k][r].y, load_at<float>(A, rowb[r]));
                pb[k][r] = make_float2(pb[k][r].y, load_at<float>(B, rowb[r]));
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int k = 0; k < D; ++k) c[0][r][0][k] = pa[k][r].x;
#pragma unroll
        for (int k = 0; k < D; ++k) c[0][r][1][k] = pa[k][r].y;
#pragma unroll
        for (int k = 0; k < D; ++k) c[1][r][0][k] = pb[k][r].x;
#pragma unroll
        for (int k = 0; k < D; ++k) c[1][r][1][k] = pb[k][r].y;
    }
}

// Frame layouts as the kernels see them (a compile-time copy of the step loop
// per layout).
constexpr int kLaySoa = 0, kLayInterleaved = 1, kLayTPair = 2;

// Gather the corner values of the cell for the frames at element offset base
// and base + frame_stride.  rowb[] are the byte offsets of the cell's rows
// (lower x corner excluded), xb0/xb1 those of its lower and upper x nodes and
// pxb that of the first node of the loaded x pair (n0-2 on a wrapped cell).
template <int D, int L>
__device__ __forceinline__ void gather_cell(const VelDev &v, long long base, const uint32_t *rowb,
                                            uint32_t xb0, uint32_t xb1, uint32_t pxb, bool wrap,
                                            float (&c)[2][CellCache<D>::R][2][D])
{
    constexpr int R = CellCache<D>::R;
    const long long fs = v.frame_stride;
    if constexpr (L == kLayTPair && D == 2) {
        // time-paired records (2D): per row the lower and upper x node, both
        // frames, in 32 contiguous bytes (a wrapped cell reads the row's extra
        // node)
        const char *__restrict__ P = reinterpret_cast<const char *>(v.ilv_u + base * 4);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t e = rowb[r] + xb0;
            const float4 q0 = load_at<float4>(P, e), q1 = load_at<float4>(P, e + 16u);
            c[0][r][0][0] = q0.x; c[0][r][0][1] = q0.y;
            c[1][r][0][0] = q0.z; c[1][r][0][1] = q0.w;
            c[0][r][1][0] = q1.x; c[0][r][1][1] = q1.y;
            c[1][r][1][0] = q1.z; c[1][r][1][1] = q1.w;
        }
    } else if constexpr (L == kLayTPair) {
        // time-paired records (3D): per row the lower and upper x node, both
        // frames, in 48 contiguous bytes (a wrapped cell reads the row's extra
        // node)
        const char *__restrict__ P = reinterpret_cast<const char *>(v.ilv_u + base * 6);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t e = rowb[r] + xb0;
            const float4 q0 = load_at<float4>(P, e), q1 = load_at<float4>(P, e + 16u),
                         q2 = load_at<float4>(P, e + 32u);
            c[0][r][0][0] = q0.x; c[0][r][0][1] = q0.y; c[0][r][0][2] = q0.z;
            c[0][r][1][0] = q1.z; c[0][r][1][1] = q1.w; c[0][r][1][2] = q2.x;
            c[1][r][0][0] = q0.w; c[1][r][0][1] = q1.x; c[1][r][0][2] = q1.y;
            c[1][r][1][0] = q2.y; c[1][r][1][1] = q2.z; c[1][r][1][2] = q2.w;
        }
    } else if constexpr (L == kLayInterleaved) {
        // interleaved layout: per (row, frame) the lower and upper node records
        const long long S = v.ilv;
        const char *__restrict__ A = reinterpret_cast<const char *>(v.ilv_u + base * S);
        const char *__restrict__ B = reinterpret_cast<const char *>(v.ilv_u + (base + fs) * S);
        if constexpr (D == 3) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t e0 = rowb[r] + xb0, e1 = rowb[r] + xb1;
                const float3 a0 = load_at<float3>(A, e0), a1 = load_at<float3>(A, e1);
                const float3 b0 = load_at<float3>(B, e0), b1 = load_at<float3>(B, e1);
                c[0][r][0][0] = a0.x; c[0][r][0][1] = a0.y; c[0][r][0][2] = a0.z;
                c[0][r][1][0] = a1.x; c[0][r][1][1] = a1.y; c[0][r][1][2] = a1.z;
                c[1][r][0][0] = b0.x; c[1][r][0][1] = b0.y; c[1][r][0][2] = b0.z;
                c[1][r][1][0] = b1.x; c[1][r][1][1] = b1.y; c[1][r][1][2] = b1.z;
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float4 qa = load_at<float4>(A, rowb[r] + pxb), qb = load_at<float4>(B, rowb[r] + pxb);
                if (wrap) {   // pair (n0-2, n0-1) -> (n0-1, 0)
                    const float2 za = load_at<float2>(A, rowb[r]), zb = load_at<float2>(B, rowb[r]);
                    qa = make_float4(qa.z, qa.w, za.x, za.y);
                    qb = make_float4(qb.z, qb.w, zb.x, zb.y);
                }
                c[0][r][0][0] = qa.x; c[0][r][0][1] = qa.y; c[0][r][1][0] = qa.z; c[0][r][1][1] = qa.w;
                c[1][r][0][0] = qb.x; c[1][r][0][1] = qb.y; c[1][r][1][0] = qb.z; c[1][r][1][1] = qb.w;
            }
        }
    } else {
        gather_cell_soa<D>(v, base, rowb, pxb, wrap, c);
    }
}

// u at the grid-index point (ph + pl): multilinear in space within frames f and
// f+1, then linear in time.  The corners of a cell come in x-adjacent pairs
// (i, i+1); on a periodic x axis the pair of the last cell wraps to node 0.
// The corner values are reused while the tracer stays in the cell and frame
// pair of its previous evaluation (cc).
template <int D, int L>
__device__ __forceinline__ void velocity(const VelDev &v, const float *ph, const float *pl,
                                         long long base, float alpha, float *out,
                                         CellCache<D> &cc)
{
    // The blends are written as explicit FMAs with contraction off, so every
    // kernel (and every frame layout) computes the same bits.
#pragma clang fp contract(off)
    int lo[3], hi[3];
    float xi[3];
#pragma unroll
    for (int a = 0; a < D; ++a) locate_s(v, a, ph[a], pl[a], lo[a], hi[a], xi[a]);
    const float a1 = alpha, a0 = 1.0f - alpha;
    const int n0 = v.n[0];
    const bool wrap = (hi[0] != lo[0] + 1);          // periodic x, last cell
    const float wx1 = xi[0], wx0 = 1.0f - xi[0];
    constexpr int R = CellCache<D>::R;
    // byte offsets within a frame array (a node's offset is its index times
    // sb[0]; hi is lo + 1 except where a periodic axis wraps to node 0)
    const uint32_t xb0 = (uint32_t)lo[0] * v.sb[0];
    const uint32_t xb1 = wrap ? 0u : xb0 + v.sb[0];
    const uint32_t pxb = wrap ? (uint32_t)(n0 - 2) * v.sb[0] : xb0;
    const uint32_t yb0 = (uint32_t)lo[1] * v.sb[1];
    const uint32_t yb1 = (hi[1] == 0) ? 0u : yb0 + v.sb[1];
    uint32_t rowb[R];
    float wr[R];
    if constexpr (D == 2) {
        const float wy1 = xi[1], wy0 = 1.0f - xi[1];
        rowb[0] = yb0; rowb[1] = yb1;
        wr[0] = wy0; wr[1] = wy1;
    } else {
        const uint32_t zb0 = (uint32_t)lo[2] * v.sb[2];
        const uint32_t zb1 = (hi[2] == 0) ? 0u : zb0 + v.sb[2];
        const float wy1 = xi[1], wy0 = 1.0f - xi[1];
        const float wz1 = xi[2], wz0 = 1.0f - xi[2];
        rowb[0] = yb0 + zb0; rowb[1] = yb1 + zb0; rowb[2] = yb0 + zb1; rowb[3] = yb1 + zb1;
        wr[0] = wy0 * wz0; wr[1] = wy1 * wz0; wr[2] = wy0 * wz1; wr[3] = wy1 * wz1;
    }
    const uint32_t key = rowb[0] + xb0;   // the cell's lower-corner offset
    if (!LCS_CELL_CACHE || cc.node != key || cc.base != base) {
        gather_cell<D, L>(v, base, rowb, xb0, xb1, pxb, wrap, cc.c);
        cc.node = key;
        cc.base = base;
    }
    // corner weights (product of the axis weights), then one FMA chain per
    // component and frame
    float w[R][2];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        w[r][0] = wr[r] * wx0;
        w[r][1] = wr[r] * wx1;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        float ua = w[0][0] * cc.c[0][0][0][k], ub = w[0][0] * cc.c[1][0][0][k];
        ua = fmaf(w[0][1], cc.c[0][0][1][k], ua);
        ub = fmaf(w[0][1], cc.c[1][0][1][k], ub);
#pragma unroll
        for (int r = 1; r < R; ++r) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                ua = fmaf(w[r][e], cc.c[0][r][e][k], ua);
                ub = fmaf(w[r][e], cc.c[1][r][e][k], ub);
            }
        }
        out[k] = fmaf(a1, ub, a0 * ua);
    }
}

template <int D>
__device__ __forceinline__ uint32_t check_point(const VelDev &v, const float *p)
{
#pragma unroll
    for (int a = 0; a < D; ++a)
        if (!isfinite(p[a])) return kNonFinite;
#pragma unroll
    for (int a = 0; a < D; ++a)
        if (!((v.periodic_mask >> a) & 1u) && !(p[a] >= v.lo[a] && p[a] <= v.hi[a])) return kOut;
    return 0;
}

// Stage increments in grid-index units: (dt/2)/h_a per axis as a two-float
// (the physical stage point x + c k sits at s(x) + (c/h) k).  The full-step
// increment dt/h_a is twice it: its two-float is exactly twice this one, and
// so is the increment formed from it, so only the half-step constants are held
// (six fewer uniform registers in the step loops).
struct IdxConsts {
    float hh[3], hl[3];
};

__device__ __forceinline__ IdxConsts idx_consts(const VelDev &v, double dt)
{
    IdxConsts c;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double h = 0.5 * dt / v.spacing_d[a];
        c.hh[a] = (float)h; c.hl[a] = (float)(h - (double)c.hh[a]);
    }
    return c;
}


// Grid-index stage point (ph + pl) = (sh + sl) + (ch_a + cl_a) k_a, or with
// twice that increment when FULL (scaling by 2 is exact).
template <int D, bool FULL = false>
__device__ __forceinline__ void stage_point_s(const float *sh, const float *sl, const float *ch,
                                              const float *cl, const float *k, float *ph, float *pl)
{
#pragma unroll
    for (int a = 0; a < D; ++a) {
        float inc = fmaf(ch[a], k[a], cl[a] * k[a]);
        if constexpr (FULL) inc = 2.0f * inc;
        two_sum(sh[a], sl[a] + inc, ph[a], pl[a]);
    }
}

// Domain test of a grid-index point: finite, and within [0, n-1] on the
// non-periodic axes (the closed domain in index units).
template <int D>
__device__ __forceinline__ uint32_t check_point_s(const VelDev &v, const float *p)
{
#pragma unroll
    for (int a = 0; a < D; ++a)
        if (!isfinite(p[a])) return kNonFinite;
#pragma unroll
    for (int a = 0; a < D; ++a)
        if (!((v.periodic_mask >> a) & 1u) && !(p[a] >= 0.0f && p[a] <= v.nf[a] - 1.0f)) return kOut;
    return 0;
}

// Integrate one tracer in place over steps n_begin <= n < n_end of classical
// RK4 from t0 with step dt, t_n = t0 + n*dt recomputed each step.  The position is carried as a
// two-float (x = xh + xl).  A stage point or new position that is non-finite
// or outside the closed domain (or a non-finite sampled velocity) rejects the
// step, freezes the tracer and returns its flag.  n_stop (if given) receives
// the index of the rejected step, or n_end: the steps before it were accepted.
template <int D, bool UNIFORM_T, int L>
__device__ uint32_t advect_steps_l(const VelDev &v, float *xh, float *xl, double t0, double dt,
                                   int n_begin, int n_end, int *n_stop)
{
    uint32_t fl = 0;
    const StepConsts sc = step_consts(dt);
    const IdxConsts ic = idx_consts(v, dt);
    CellCache<D> cc;
    int n = n_begin;
    for (; n < n_end; ++n) {
        const double t = t0 + (double)n * dt;
        long long b1, b2, b4;
        float al1, al2, al4;
        if constexpr (UNIFORM_T) {
            frame_at_uniform(v, t, b1, al1);
            frame_at_uniform(v, t + 0.5 * dt, b2, al2);
            frame_at_uniform(v, t + dt, b4, al4);
        } else {
            frame_at(v, t, b1, al1);
            frame_at(v, t + 0.5 * dt, b2, al2);
            frame_at(v, t + dt, b4, al4);
        }
        // the position in grid-index units once per step; the stage points
        // are formed there directly
        float k1[3], k2[3], k3[3], k4[3], sh[3], sl[3], ph[3], pl[3];
#pragma unroll
        for (int a = 0; a < D; ++a) to_index(v, a, xh[a], xl[a], sh[a], sl[a]);

        velocity<D, L>(v, sh, sl, b1, al1, k1, cc);
        if (!finite_vec<D>(k1)) { fl = kNonFinite; break; }
        stage_point_s<D>(sh, sl, ic.hh, ic.hl, k1, ph, pl);
        if ((fl = check_point_s<D>(v, ph))) break;

        velocity<D, L>(v, ph, pl, b2, al2, k2, cc);
        if (!finite_vec<D>(k2)) { fl = kNonFinite; break; }
        stage_point_s<D>(sh, sl, ic.hh, ic.hl, k2, ph, pl);
        if ((fl = check_point_s<D>(v, ph))) break;

        velocity<D, L>(v, ph, pl, b2, al2, k3, cc);
        if (!finite_vec<D>(k3)) { fl = kNonFinite; break; }
        stage_point_s<D, true>(sh, sl, ic.hh, ic.hl, k3, ph, pl);
        if ((fl = check_point_s<D>(v, ph))) break;

        velocity<D, L>(v, ph, pl, b4, al4, k4, cc);
        if (!finite_vec<D>(k4)) { fl = kNonFinite; break; }

        // (xh, xl) <- (xh, xl) + dt/6 (k1 + 2k2 + 2k3 + k4)
        float nh[3], nl[3];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const float sum = (k1[a] + k4[a]) + 2.0f * (k2[a] + k3[a]);
            const float inc = fmaf(sc.sh, sum, sc.sl * sum);
            two_sum(xh[a], xl[a] + inc, nh[a], nl[a]);
        }
        if ((fl = check_point<D>(v, nh))) break;
#pragma unroll
        for (int a = 0; a < D; ++a) { xh[a] = nh[a]; xl[a] = nl[a]; }
    }
    if (n_stop) *n_stop = n;
    return fl;
}

// The frame layout is fixed for a launch: each layout gets its own copy of the
// step loop (and of the cell cache's registers).
template <int D, bool UNIFORM_T = true>
__device__ uint32_t advect_steps(const VelDev &v, float *xh, float *xl, double t0, double dt,
                                 int n_begin, int n_end, int *n_stop = nullptr)
{
    if (v.ilv == 2 * D)   // time-paired records (interleaved records have dim or 4 floats, 4 only in 3D)
        return advect_steps_l<D, UNIFORM_T, kLayTPair>(v, xh, xl, t0, dt, n_begin, n_end, n_stop);
    if (v.ilv)
        return advect_steps_l<D, UNIFORM_T, kLayInterleaved>(v, xh, xl, t0, dt, n_begin, n_end, n_stop);
    return advect_steps_l<D, UNIFORM_T, kLaySoa>(v, xh, xl, t0, dt, n_begin, n_end, n_stop);
}

// UNIFORM_T: every lane of the wave integrates from the same t0 (grid,
// batched, re-bundled and check launches); per-point start times use false.
template <int D, bool UNIFORM_T = true>
__device__ uint32_t advect_tracer(const VelDev &v, float *xh, float *xl, double t0, double dt,
                                  int nsteps)
{
    const uint32_t fl = check_point<D>(v, xh);
    if (fl) return fl;
    return advect_steps<D, UNIFORM_T>(v, xh, xl, t0, dt, 0, nsteps);
}

// Velocity-cell index of a returned FP32 position, in FP64 without
// contraction: per axis s = (x - origin)/h, then the locate rule.  -1 for a
// non-finite position.
template <int D>
__device__ long long cell_index(const VelDev &v, const float *x)
{
#pragma clang fp contract(off)
    long long idx = 0, stride = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double xd = (double)x[a];
        if (!isfinite(xd)) return -1;
        const long long n = v.n[a];
        double s = (xd - v.origin_d[a]) / v.spacing_d[a];
        long long i;
        if ((v.periodic_mask >> a) & 1u) {
            const double nd = (double)n;
            s = s - nd * floor(s / nd);
            s = fmin(fmax(s, -1.0), nd + 1.0);
            i = (long long)floor(s);
            if (i >= n) i = 0;
            if (i < 0) i = 0;
        } else {
            s = fmin(fmax(s, -1.0), (double)n);
            i = (long long)floor(s);
            if (i > n - 2) i = n - 2;
            if (i < 0) i = 0;
        }
        idx += i * stride;
        stride *= n;
    }
    return idx;
}

// Advect the seed with integer coordinates sc from t0 and write its outputs at
// linear index s of the given output arrays.
template <int D>
__device__ __forceinline__ void advect_seed(const VelDev &v, const SeedTiling &g, const int *sc,
                                            long long s, double t0, double dt, int nsteps,
                                            long long ns, float *xf, long long *cell,
                                            uint8_t *flags)
{
    // seed position, carried exactly (to FP64 rounding) as a two-float
    float xh[3], xl[3], x[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double x0 = g.s_origin[a] + (double)sc[a] * g.s_spacing[a];
        xh[a] = (float)x0;
        xl[a] = (float)(x0 - (double)xh[a]);
    }
    const uint32_t fl = advect_tracer<D>(v, xh, xl, t0, dt, nsteps);
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = xh[a] + xl[a];
#pragma unroll
    for (int a = 0; a < D; ++a) xf[a * ns + s] = x[a];
    if (cell) cell[s] = cell_index<D>(v, x);
    if (flags) flags[s] = (uint8_t)fl;
}

template <int D>
__global__ LCS_RK4_BOUNDS void advect_grid_kernel(AdvectArgs A)
{
    const int m = xcd_remap((int)blockIdx.x, A.g.n_blocks);
    int sc[3];
    const long long s = seed_of<D>(A.g, m, threadIdx.x, sc);
    if (s < 0) return;
    advect_seed<D>(A.v, A.g, sc, s, A.t0, A.dt, A.nsteps, A.ns, A.xf, A.cell, A.flags);
}

// ---------------------------------------------------------------------------
// Adams-Bashforth multistep advection (the Flow Map filter admits multistep
// methods, Sec. 2): one velocity evaluation per step instead of RK4's four.
// x_{n+1} = x_n + (dt/den) sum_j num_j f_{n-j} with integer numerators
// (3, -1)/2, (23, -16, 5)/12, (55, -59, 37, -9)/24, the combination formed in
// FP32 (exact integer weights) and scaled by dt/den as a two-float.  The first
// S-1 steps are classical RK4 steps whose first stage is f_n.  The past
// velocities stay in registers.
// ---------------------------------------------------------------------------
template <int S>
__device__ __forceinline__ float ab_num(int j)
{
    if constexpr (S == 2) return j == 0 ? 3.0f : -1.0f;
    else if constexpr (S == 3) return j == 0 ? 23.0f : (j == 1 ? -16.0f : 5.0f);
    else return j == 0 ? 55.0f : (j == 1 ? -59.0f : (j == 2 ? 37.0f : -9.0f));
}

template <int S>
constexpr double ab_den() { return S == 2 ? 2.0 : (S == 3 ? 12.0 : 24.0); }

// Steps n_begin <= n < n_end; hist[j] = f_{n-1-j} on entry and is updated, so
// an integration can be resumed from a saved (position, history) state.
template <int D, int S, int L>
__device__ uint32_t advect_steps_ab_l(const VelDev &v, float *xh, float *xl, float (*hist)[3],
                                      double t0, double dt, int n_begin, int n_end)
{
    uint32_t fl = 0;
    const StepConsts sc = step_consts(dt);
    const double cab = dt / ab_den<S>();
    const float ch = (float)cab, cl = (float)(cab - (double)ch);
    const IdxConsts ic = idx_consts(v, dt);
    CellCache<D> cc;
    for (int n = n_begin; n < n_end; ++n) {
        const double t = t0 + (double)n * dt;
        long long b1;
        float al1;
        frame_at_uniform(v, t, b1, al1);
        float k1[3], sh[3], sl[3];
#pragma unroll
        for (int a = 0; a < D; ++a) to_index(v, a, xh[a], xl[a], sh[a], sl[a]);
        velocity<D, L>(v, sh, sl, b1, al1, k1, cc);
        if (!finite_vec<D>(k1)) { fl = kNonFinite; break; }
        float nh[3], nl[3];
        if (n < S - 1) {
            long long b2, b4;
            float al2, al4;
            frame_at_uniform(v, t + 0.5 * dt, b2, al2);
            frame_at_uniform(v, t + dt, b4, al4);
            float k2[3], k3[3], k4[3], ph[3], pl[3];
            stage_point_s<D>(sh, sl, ic.hh, ic.hl, k1, ph, pl);
            if ((fl = check_point_s<D>(v, ph))) break;
            velocity<D, L>(v, ph, pl, b2, al2, k2, cc);
            if (!finite_vec<D>(k2)) { fl = kNonFinite; break; }
            stage_point_s<D>(sh, sl, ic.hh, ic.hl, k2, ph, pl);
            if ((fl = check_point_s<D>(v, ph))) break;
            velocity<D, L>(v, ph, pl, b2, al2, k3, cc);
            if (!finite_vec<D>(k3)) { fl = kNonFinite; break; }
            stage_point_s<D, true>(sh, sl, ic.hh, ic.hl, k3, ph, pl);
            if ((fl = check_point_s<D>(v, ph))) break;
            velocity<D, L>(v, ph, pl, b4, al4, k4, cc);
            if (!finite_vec<D>(k4)) { fl = kNonFinite; break; }
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const float sum = (k1[a] + k4[a]) + 2.0f * (k2[a] + k3[a]);
                const float inc = fmaf(sc.sh, sum, sc.sl * sum);
                two_sum(xh[a], xl[a] + inc, nh[a], nl[a]);
            }
        } else {
#pragma unroll
            for (int a = 0; a < D; ++a) {
                float sum = ab_num<S>(0) * k1[a];
#pragma unroll
                for (int j = 1; j < S; ++j) sum = fmaf(ab_num<S>(j), hist[j - 1][a], sum);
                const float inc = fmaf(ch, sum, cl * sum);
                two_sum(xh[a], xl[a] + inc, nh[a], nl[a]);
            }
        }
        if ((fl = check_point<D>(v, nh))) break;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            xh[a] = nh[a];
            xl[a] = nl[a];
            hist[2][a] = hist[1][a];
            hist[1][a] = hist[0][a];
            hist[0][a] = k1[a];
        }
    }
    return fl;
}

template <int D, int S>
__device__ uint32_t advect_steps_ab(const VelDev &v, float *xh, float *xl, float (*hist)[3],
                                    double t0, double dt, int n_begin, int n_end)
{
    if (v.ilv == 2 * D) return advect_steps_ab_l<D, S, kLayTPair>(v, xh, xl, hist, t0, dt, n_begin, n_end);
    if (v.ilv) return advect_steps_ab_l<D, S, kLayInterleaved>(v, xh, xl, hist, t0, dt, n_begin, n_end);
    return advect_steps_ab_l<D, S, kLaySoa>(v, xh, xl, hist, t0, dt, n_begin, n_end);
}

template <int D, int S>
__global__ LCS_AB_BOUNDS void advect_ab_grid_kernel(AdvectArgs A)
{
    const int m = xcd_remap((int)blockIdx.x, A.g.n_blocks);
    int sc[3];
    const long long s = seed_of<D>(A.g, m, threadIdx.x, sc);
    if (s < 0) return;
    float xh[3], xl[3], x[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double x0 = A.g.s_origin[a] + (double)sc[a] * A.g.s_spacing[a];
        xh[a] = (float)x0;
        xl[a] = (float)(x0 - (double)xh[a]);
    }
    uint32_t fl = check_point<D>(A.v, xh);
    float hist[3][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
    if (!fl) fl = advect_steps_ab<D, S>(A.v, xh, xl, hist, A.t0, A.dt, 0, A.nsteps);
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = xh[a] + xl[a];
#pragma unroll
    for (int a = 0; a < D; ++a) A.xf[a * A.ns + s] = x[a];
    if (A.cell) A.cell[s] = cell_index<D>(A.v, x);
    if (A.flags) A.flags[s] = (uint8_t)fl;
}

// Auxiliary points (Sec. 2 Seed and Cauchy-Green filters): a block advects
// point q = 2b + side of every seed of one tile, which starts at
// x0 - delta_b e_b (side 0) or x0 + delta_b e_b (side 1), formed in FP64 and
// carried as a two-float.  The 2*dim blocks of a tile are consecutive in the
// XCD-remapped order, so they run together on one XCD and share its L2 (their
// trajectories stay within about delta of each other).  Outputs keep the
// two-float (hi, lo) so that the gradient can difference exact FP64 positions.
template <int D>
__global__ LCS_RK4_BOUNDS void advect_aux_kernel(AuxArgs A)
{
    const int r = xcd_remap((int)blockIdx.x, A.a.g.n_blocks * 2 * D);
    const int m = r / (2 * D);
    const int q = r - m * (2 * D);
    const int b = q >> 1, side = q & 1;
    int sc[3];
    const long long s = seed_of<D>(A.a.g, m, threadIdx.x, sc);
    if (s < 0) return;
    float xh[3], xl[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double x0 = A.a.g.s_origin[a] + (double)sc[a] * A.a.g.s_spacing[a];
        if (a == b) x0 = side ? x0 + A.delta[a] : x0 - A.delta[a];
        xh[a] = (float)x0;
        xl[a] = (float)(x0 - (double)xh[a]);
    }
    const uint32_t fl = advect_tracer<D>(A.a.v, xh, xl, A.a.t0, A.a.dt, A.a.nsteps);
    const long long ns = A.a.ns;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        A.xa_hi[((long long)a * 2 * D + q) * ns + s] = xh[a];
        A.xa_lo[((long long)a * 2 * D + q) * ns + s] = xl[a];
    }
    if (A.a.flags) A.a.flags[(long long)q * ns + s] = (uint8_t)fl;
}

// Time-resolved flow map (Sec. 3.1: the CG tensor at any step of the
// interval): the grid kernel's integration, writing the position and flag of
// every tracer after each listed step count, and the number of steps it took
// before it froze.
template <int D>
__global__ LCS_RK4_BOUNDS void advect_snap_kernel(SnapArgs A)
{
    const int m = xcd_remap((int)blockIdx.x, A.a.g.n_blocks);
    int sc[3];
    const long long s = seed_of<D>(A.a.g, m, threadIdx.x, sc);
    if (s < 0) return;
    float xh[3], xl[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double x0 = A.a.g.s_origin[a] + (double)sc[a] * A.a.g.s_spacing[a];
        xh[a] = (float)x0;
        xl[a] = (float)(x0 - (double)xh[a]);
    }
    uint32_t fl = check_point<D>(A.a.v, xh);
    int nacc = 0, n = 0;
    const long long ns = A.a.ns;
    // from one listed step count to the next in one call, so the tracer's cell
    // cache carries across the steps of a stretch
    for (int k = 0; k < A.n_snap; ++k) {
        const int nk = A.steps[k];
        if (!fl && nk > n) {
            int stop = nk;
            fl = advect_steps<D, true>(A.a.v, xh, xl, A.a.t0, A.a.dt, n, nk, &stop);
            nacc = stop;
        }
        n = nk;
#pragma unroll
        for (int a = 0; a < D; ++a) A.xf[((long long)k * D + a) * ns + s] = xh[a] + xl[a];
        if (A.flags) A.flags[(long long)k * ns + s] = (uint8_t)fl;
    }
    if (A.steps_done) A.steps_done[s] = nacc;
}

// Early evaluation: re-advect the stencil members of listed seeds for their
// n_s steps.  Work item w = entry * 7 + slot; slot 0 is the seed, slot
// 1 + 2b + side its lower (side 0) / upper neighbour along b.  Slots past the
// grid's dimension or past a non-periodic edge have no member.  Positions
// are written in FP64 (two-float sum).
template <int D>
__global__ LCS_RK4_BOUNDS void early_advect_kernel(EarlyAdvArgs A, int first, int count)
{
    const long long w = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int e = (int)(w / 7), slot = (int)(w % 7);
    if (e >= count) return;
    const long long s = A.list[2 * (first + e)];
    const int nsd = A.list[2 * (first + e) + 1];
    int c[3] = {(int)(s % A.n[0]), (int)((s / A.n[0]) % A.n[1]),
                (int)(s / ((long long)A.n[0] * A.n[1]))};
    if (slot > 0) {
        const int b = (slot - 1) >> 1, dir = ((slot - 1) & 1) ? 1 : -1;
        if (b >= D) return;
        int j = c[b] + dir;
        if ((A.periodic_mask >> b) & 1u) j = (j + A.n[b]) % A.n[b];
        else if (j < 0 || j >= A.n[b]) return;
        c[b] = j;
    }
    float xh[3], xl[3];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double x0 = A.s_origin[a] + (double)c[a] * A.s_spacing[a];
        xh[a] = (float)x0;
        xl[a] = (float)(x0 - (double)xh[a]);
    }
    (void)advect_tracer<D>(A.v, xh, xl, A.t0, A.dt, nsd);
    double *P = A.pos + ((long long)e * 7 + slot) * 3;
#pragma unroll
    for (int a = 0; a < D; ++a) P[a] = (double)xh[a] + (double)xl[a];
}

// Structure-of-arrays frames -> interleaved (S floats per node; a 4th float
// of 3D records is 0), frames f_first .. f_first + f_count - 1.
__global__ __launch_bounds__(256) void interleave_kernel(int dim, int S, const float *u0,
                                                        const float *u1, const float *u2,
                                                        long long n, long long off, float *out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float *o = out + i * S;
    o[0] = u0[off + i];
    o[1] = u1[off + i];
    if (dim == 3) o[2] = u2[off + i];
    if (S == 4) o[3] = 0.0f;
}

// Time-paired records (2*D floats: the D components of frame p, then those of
// frame p + 1): one thread per record q on the grid with n0 + 1 nodes per row
// (the last repeating node 0 of the row), for the kTPairRun consecutive pairs
// p = pair0 + kTPairRun*blockIdx.y .. (< pairs) (frames f_first + p and
// f_first + p + 1): the frame two neighbouring pairs share stays in
// registers, so each frame is read once per run instead of twice.  The
// records of one pair number fewer than 2^28 (a frame-pair block is limited
// to 4 GiB), so the index arithmetic within a pair is 32-bit.  In 2D, n2 = 1
// and u2 is not read.
constexpr int kTPairRun = 8;

template <int D>
__global__ __launch_bounds__(256) void interleave_tpair_kernel(const float *__restrict__ u0,
                                                               const float *__restrict__ u1,
                                                               const float *__restrict__ u2,
                                                               int n0, int n1, int n2,
                                                               long long f_first, long long pair0,
                                                               long long pairs,
                                                               float *__restrict__ out)
{
    const uint32_t w = (uint32_t)n0 + 1u;
    const uint32_t per_pair = w * (uint32_t)n1 * (uint32_t)n2;
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= per_pair) return;
    const long long p0 = pair0 + (long long)kTPairRun * blockIdx.y;
    const long long p1 = (pairs - p0 < kTPairRun) ? pairs : p0 + kTPairRun;
    const uint32_t row = q / w;                    // j + n1*k
    const uint32_t i = q - row * w;
    const long long nodes = (long long)n0 * n1 * n2;
    const long long node = (long long)row * n0 + (i == (uint32_t)n0 ? 0u : i);
    long long a = (f_first + p0) * nodes + node;
    float x0 = u0[a], y0 = u1[a], z0 = (D == 3) ? u2[a] : 0.0f;
    for (long long p = p0; p < p1; ++p) {
        a += nodes;
        const float x1 = u0[a], y1 = u1[a], z1 = (D == 3) ? u2[a] : 0.0f;
        if constexpr (D == 3) {
            float2 *o = reinterpret_cast<float2 *>(out + (p * (long long)per_pair + q) * 6);
            o[0] = make_float2(x0, y0);
            o[1] = make_float2(z0, x1);
            o[2] = make_float2(y1, z1);
        } else {
            *reinterpret_cast<float4 *>(out + (p * (long long)per_pair + q) * 4) =
                make_float4(x0, y0, x1, y1);
        }
        x0 = x1;
        y0 = y1;
        z0 = z1;
    }
}

__global__ void reset_counter_kernel(int *counter)
{
    if (threadIdx.x < kBatchCounters) counter[threadIdx.x] = 0;
}

// Persistent batched advection.  The seed tiles (in Morton order) are split
// into 8 contiguous runs, one per XCD (blocks are dealt round-robin to the
// XCDs, so block b works on run b % 8): each XCD then gathers from one
// compact eighth of the domain, which its L2 holds, instead of every XCD
// reading whole frames.  A block repeatedly claims the next (window, tile) item
// of its run from the run's own counter, windows in start-time order and,
// within a window, tiles along the Morton curve.  All lanes of a block leave
// the loop together once the run's counter passes its item count.
template <int D>
__global__ __launch_bounds__(256) void advect_batched_kernel(BatchArgs A)
{
    __shared__ int s_item;
    const int x = blockIdx.x % kBatchCounters;
    const int nb = A.g.n_blocks, q8 = nb / kBatchCounters, r8 = nb % kBatchCounters;
    const int run = q8 + (x < r8 ? 1 : 0);                 // tiles of this XCD's run
    const int first = x * q8 + min(x, r8);                 // its first tile
    const int items = A.n_windows * run;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(A.counter + x, 1);
        __syncthreads();
        const int q = s_item;
        __syncthreads();
        if (q >= items) break;
        const int k = q / run;
        const int m = first + (q - k * run);
        const WindowDev w = A.win[k];
        int sc[3];
        const long long s = seed_of<D>(A.g, m, threadIdx.x, sc);
        if (s >= 0) {
            const long long off = (long long)w.out_index * A.ns;
            advect_seed<D>(A.v, A.g, sc, s, w.t0, A.dt, w.nsteps, A.ns, A.xf + D * off,
                           A.cell ? A.cell + off : nullptr, A.flags ? A.flags + off : nullptr);
        }
    }
}

template <int D>
__global__ __launch_bounds__(256) void advect_points_kernel(AdvectArgs A)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.ns) return;
    float x[3], xl[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = A.x0[a * A.ns + p];
    const double t0 = A.t0v[p];
    const double t1 = t0 + A.T;
    uint32_t fl;
    // no extrapolation in time: the whole interval must lie in the frame span
    if (!(t0 >= A.v.t_first && t0 <= A.v.t_last && t1 >= A.v.t_first && t1 <= A.v.t_last)) {
        fl = kTimeOut;
    } else {
        fl = advect_tracer<D, false>(A.v, x, xl, t0, A.dt, A.nsteps);
#pragma unroll
        for (int a = 0; a < D; ++a) x[a] = x[a] + xl[a];
    }
#pragma unroll
    for (int a = 0; a < D; ++a) A.xf[a * A.ns + p] = x[a];
    if (A.cell) A.cell[p] = cell_index<D>(A.v, x);
    if (A.flags) A.flags[p] = (uint8_t)fl;
}

// ---------------------------------------------------------------------------
// Surrogate check samples and tile fallback (3D).  Check tiles are aligned
// 16 x 16 x 8 blocks of seeds (2048); within a tile the seeds with local
// linear index 0, 100, 200, ... (about 1 %) are advected with RK4 over the
// whole window and compared with the surrogate's positions.
// ---------------------------------------------------------------------------
constexpr int kCtX = 16, kCtY = 16, kCtZ = 8, kCtSeeds = kCtX * kCtY * kCtZ, kCtStride = 100;
constexpr int kCtSamples = (kCtSeeds + kCtStride - 1) / kCtStride;

__global__ __launch_bounds__(256) void clear_check_kernel(float *tile_err, uint8_t *tile_fail,
                                                          int *n_fail, long long n_tiles)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_tiles) {
        tile_err[i] = 0.0f;
        tile_fail[i] = 0;
    }
    if (i == 0) *n_fail = 0;
}

__global__ __launch_bounds__(256) void check_kernel(CheckArgs A)
{
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= A.n_tiles * kCtSamples) return;
    const long long tile = id / kCtSamples;
    const int q = (int)(id % kCtSamples) * kCtStride;
    const int tx = (int)(tile % A.ct[0]);
    const int ty = (int)((tile / A.ct[0]) % A.ct[1]);
    const int tz = (int)(tile / ((long long)A.ct[0] * A.ct[1]));
    int sc[3] = {tx * kCtX + q % kCtX, ty * kCtY + (q / kCtX) % kCtY, tz * kCtZ + q / (kCtX * kCtY)};
    if (sc[0] >= A.g.sn[0] || sc[1] >= A.g.sn[1] || sc[2] >= A.g.sn[2]) return;
    const long long s = (long long)sc[0] + (long long)A.g.sn[0] * ((long long)sc[1] +
                        (long long)A.g.sn[1] * (long long)sc[2]);
    float xh[3], xl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double x0 = A.g.s_origin[a] + (double)sc[a] * A.g.s_spacing[a];
        xh[a] = (float)x0;
        xl[a] = (float)(x0 - (double)xh[a]);
    }
    const uint32_t fl = advect_tracer<3>(A.v, xh, xl, A.t0, A.dt, A.nsteps);
    float err2 = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float d = (xh[a] + xl[a]) - A.xf[a * A.ns + s];
        err2 += d * d;
    }
    float err = sqrtf(err2);
    if (fl || !(err == err)) err = INFINITY;   // a flagged or NaN check sample fails its tile
    // non-negative floats order like their bit patterns
    atomicMax(reinterpret_cast<unsigned int *>(A.tile_err) + tile, __float_as_uint(err));
}

__global__ __launch_bounds__(256) void mark_kernel(const float *tile_err, float tol, uint8_t *tile_fail,
                                                   int *n_fail, long long n_tiles)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_tiles) return;
    const bool bad = !(tile_err[i] <= tol);
    tile_fail[i] = bad ? 1 : 0;
    if (bad) atomicAdd(n_fail, 1);
}

// Plain RK4 for every seed of the failing check tiles: a check tile is 8
// workgroup tiles of 8 x 8 x 4 seeds (2 x 2 x 2).
__global__ __launch_bounds__(256) void advect_tiles_kernel(AdvectArgs A, const uint8_t *tile_fail,
                                                           int ct0, int ct1)
{
    const long long b = blockIdx.x;
    const long long tile = b / 8;
    if (!tile_fail[tile]) return;
    const int sub = (int)(b % 8);
    const int tx = (int)(tile % ct0), ty = (int)((tile / ct0) % ct1), tz = (int)(tile / ((long long)ct0 * ct1));
    const SeedTiling &g = A.g;
    const int t = threadIdx.x;
    const int w = t / kWave, l = t % kWave;
    int sc[3];
    sc[0] = tx * kCtX + (sub % 2) * 8 + (w % 2) * 4 + l % 4;
    sc[1] = ty * kCtY + ((sub / 2) % 2) * 8 + (w / 2) * 4 + (l / 4) % 4;
    sc[2] = tz * kCtZ + (sub / 4) * 4 + l / 16;
    if (sc[0] >= g.sn[0] || sc[1] >= g.sn[1] || sc[2] >= g.sn[2]) return;
    const long long s = (long long)sc[0] + (long long)g.sn[0] * ((long long)sc[1] +
                        (long long)g.sn[1] * (long long)sc[2]);
    advect_seed<3>(A.v, g, sc, s, A.t0, A.dt, A.nsteps, A.ns, A.xf, A.cell, A.flags);
}

// ---------------------------------------------------------------------------
// Re-bundled advection kernels
// ---------------------------------------------------------------------------

// Morton key of the coarse bin holding the point (periodic axes wrap, others
// clamp; NaN lands in bin 0).
template <int D>
__device__ __forceinline__ uint32_t bin_key(const VelDev &v, const SortKeys &k, const float *x)
{
    int b[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        float q = (x[a] - k.origin[a]) * k.inv_bin[a];
        const float nbf = (float)k.nb[a];
        if ((v.periodic_mask >> a) & 1u) q = q - nbf * floorf(q / nbf);
        q = fminf(fmaxf(q, 0.0f), nbf - 1.0f);
        b[a] = (int)q;
    }
    uint32_t key = 0;
    int pos = 0;
    for (int l = 0; l < k.max_bits; ++l)
#pragma unroll
        for (int a = 0; a < D; ++a)
            if (l < k.bits[a]) key |= (uint32_t)((b[a] >> l) & 1) << (pos++);
    return key;
}

// counts[key] += 1 for every active lane, one atomic per run of consecutive
// active lanes with equal keys (tracers that stay together keep landing in the
// same bin, and same-address atomics from one wave serialise).  Returns the
// lane's rank among the slots of its key: the counter's old value plus the
// lane's rank in its run (kept, so the permutation needs no second pass of
// atomics).
__device__ __forceinline__ uint32_t run_atomic_inc(uint32_t *counts, uint32_t key)
{
    const uint64_t act = __ballot(1);
    const int lane = (int)__lane_id();
    const uint32_t prev = (uint32_t)__shfl_up((int)key, 1);
    const bool start = lane == 0 || !((act >> (lane - 1)) & 1ull) || prev != key;
    const uint64_t starts = __ballot(start);
    const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);   // lanes <= lane
    const int s0 = 63 - __clzll(starts & upto);                              // my run's first lane
    const uint64_t later = starts & ~upto;
    const int s1 = later ? __ffsll((long long)later) - 1 : 64;               // next run's first lane
    const uint64_t run = ((s1 == 64) ? ~0ull : ((1ull << s1) - 1ull)) & ~((1ull << s0) - 1ull);
    uint32_t base = 0;
    if (lane == s0) base = atomicAdd(&counts[key], (uint32_t)__popcll(act & run));
    base = (uint32_t)__shfl((int)base, s0);
    return base + (uint32_t)(lane - s0);
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *p, long long n, uint32_t v)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void fill_u8_kernel(uint8_t *p, long long n, uint8_t v)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// State of every seed in natural order, its flag for a start outside the
// domain, its key and the bin histogram.
template <int D>
__global__ __launch_bounds__(256) void rebundle_init_kernel(SegmentArgs A)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    const SeedTiling &g = A.g;
    // a seed, or auxiliary point q = 2b + side of seed s (side 0: x0 - delta_b e_b)
    const int q = A.aux ? (int)(p / A.ns_seeds) : -1;
    const long long sd = A.aux ? p - (long long)q * A.ns_seeds : p;
    const long long c[3] = {sd % g.sn[0], (sd / g.sn[0]) % g.sn[1], sd / ((long long)g.sn[0] * g.sn[1])};
    float xh[3] = {0, 0, 0}, xl[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double x0 = g.s_origin[a] + (double)c[a] * g.s_spacing[a];
        if (a == (q >> 1)) x0 = (q & 1) ? x0 + A.delta[a] : x0 - A.delta[a];
        xh[a] = (float)x0;
        xl[a] = (float)(x0 - (double)xh[a]);
        A.st.xh[a][p] = xh[a];
        A.st.xl[a][p] = xl[a];
    }
    A.st.idx[p] = (int)p;
    A.st.flag[p] = (uint8_t)check_point<D>(A.v, xh);
    if (A.st.hist[0])
#pragma unroll
        for (int q = 0; q < 3 * D; ++q) A.st.hist[q][p] = 0.0f;
    const uint32_t key = bin_key<D>(A.v, A.sk, xh);
    A.sk.keys[p] = key;
    A.sk.rank[p] = run_atomic_inc(A.sk.counts, key);
}

// Steps [n_begin, n_end) for every tracer slot p of the sorted order, whose
// state is read from slot perm[p] of the previous order; then either the
// outputs (last segment) or the state at slot p of the other buffer plus its
// new key, the histogram and the slot's rank within its key.
template <int D, int S>
__global__ __launch_bounds__(256, S == 0 ? LCS_RK4_MIN_WAVES : 1) void rebundle_segment_kernel(SegmentArgs A)
{
    const int nblocks = (int)gridDim.x;
    const long long p = (long long)xcd_remap((int)blockIdx.x, nblocks) * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    const long long r = A.sk.perm[p];
    if (r >= A.n) return;   // cannot happen: the permutation is a bijection of [0, n)
    float xh[3] = {0, 0, 0}, xl[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        xh[a] = A.st.xh[a][r];
        xl[a] = A.st.xl[a][r];
    }
    uint32_t fl = A.st.flag[r];
    const int sid = A.st.idx[r];
    float hist[3][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
    if constexpr (S > 0) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int a = 0; a < D; ++a) hist[j][a] = A.st.hist[j * D + a][r];
        if (!fl) fl = advect_steps_ab<D, S>(A.v, xh, xl, hist, A.t0, A.dt, A.n_begin, A.n_end);
    } else {
        if (!fl) fl = advect_steps<D>(A.v, xh, xl, A.t0, A.dt, A.n_begin, A.n_end);
    }
    if (A.last) {
        const long long s = sid;
        float x[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < D; ++a) {
            x[a] = xh[a] + xl[a];
            if (A.xf_lo) {
                A.xf[a * A.n + s] = xh[a];
                A.xf_lo[a * A.n + s] = xl[a];
            } else {
                A.xf[a * A.n + s] = x[a];
            }
        }
        if (A.cell) A.cell[s] = cell_index<D>(A.v, x);
        if (A.flags) A.flags[s] = (uint8_t)fl;
        return;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        A.out.xh[a][p] = xh[a];
        A.out.xl[a][p] = xl[a];
    }
    A.out.flag[p] = (uint8_t)fl;
    A.out.idx[p] = sid;
    if constexpr (S > 0) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int a = 0; a < D; ++a) A.out.hist[j * D + a][p] = hist[j][a];
    }
    const uint32_t key = bin_key<D>(A.v, A.sk, xh);
    A.sk.keys[p] = key;
    A.sk.rank[p] = run_atomic_inc(A.sk.counts, key);
}

// Exclusive scan of the counts: blocks of 1024 (4 per thread), block totals,
// one block scanning the totals, then the block offsets added back.
constexpr int kScanBlock = 1024;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t add = (t >= off) ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    total = sh[255];
    const uint32_t incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(256) void scan_blocks_kernel(uint32_t *data, long long n, uint32_t *sums)
{
    __shared__ uint32_t sh[256];
    const long long base = (long long)blockIdx.x * kScanBlock + 4LL * threadIdx.x;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        v[e] = (base + e < n) ? data[base + e] : 0u;
        s += v[e];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (base + e < n) data[base + e] = run;
        run += v[e];
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void scan_sums_kernel(uint32_t *sums, long long nb)
{
    __shared__ uint32_t sh[256];
    uint32_t carry = 0;
    for (long long base = 0; base < nb; base += 256) {
        const long long i = base + threadIdx.x;
        const uint32_t v = (i < nb) ? sums[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(v, sh, total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(256) void scan_add_kernel(uint32_t *data, long long n, const uint32_t *sums)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) data[i] += sums[i / kScanBlock];
}

// Slot p goes to sorted slot q = offset[key] + (its rank among the bin's
// arrivals): perm[q] = p.  The next segment reads the state through perm, so
// only the 4-byte slot index moves here, not the tracer state.
__global__ __launch_bounds__(256) void permute_kernel(SortKeys sk, long long n)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    // counts holds each key's first sorted slot (the scanned histogram) and
    // rank the slot's place among its key's slots, taken when the histogram
    // was counted: together a bijection onto [0, n)
    const long long q = (long long)sk.counts[sk.keys[p]] + sk.rank[p];
    if (q >= n) return;   // cannot happen when the histogram matches the keys
    sk.perm[q] = (uint32_t)p;
}

}  // namespace

long long exclusive_scan_sums_needed(long long n) { return (n + kScanBlock - 1) / kScanBlock; }

// In-place exclusive prefix sum of n uint32 values; block_sums holds
// exclusive_scan_sums_needed(n) values of scratch.
hipError_t launch_exclusive_scan_u32(uint32_t *data, long long n, uint32_t *block_sums,
                                     hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const long long nb = exclusive_scan_sums_needed(n);
    hipLaunchKernelGGL(scan_blocks_kernel, dim3((unsigned)nb), dim3(256), 0, s, data, n, block_sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(256), 0, s, block_sums, nb);
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, data,
                       n, block_sums);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, long long n, uint32_t v, hipStream_t s)
{
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, long long n, uint8_t v, hipStream_t s)
{
    hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_rebundle_init(int dim, const SegmentArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    if (dim == 2) hipLaunchKernelGGL(rebundle_init_kernel<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(rebundle_init_kernel<3>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rebundle_segment(int dim, const SegmentArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    char name[64];
    snprintf(name, sizeof(name), "rebundle_segment_kernel<%d, %d>", dim, a.order);
    LaunchTimer timer(name, s);
    if (dim == 2) {
        switch (a.order) {
        case 2: hipLaunchKernelGGL((rebundle_segment_kernel<2, 2>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((rebundle_segment_kernel<2, 3>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((rebundle_segment_kernel<2, 4>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((rebundle_segment_kernel<2, 0>), grid, block, 0, s, a);
        }
    } else {
        switch (a.order) {
        case 2: hipLaunchKernelGGL((rebundle_segment_kernel<3, 2>), grid, block, 0, s, a); break;
        case 3: hipLaunchKernelGGL((rebundle_segment_kernel<3, 3>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((rebundle_segment_kernel<3, 4>), grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL((rebundle_segment_kernel<3, 0>), grid, block, 0, s, a);
        }
    }
    timer.stop(s);
    return hipGetLastError();
}

// counts (histogram) -> exclusive offsets -> the permutation of the slots;
// then the counts are cleared for the next histogram.
hipError_t launch_rebundle_sort(const SegmentArgs &a, hipStream_t s)
{
    const long long nk = a.sk.n_keys;
    const hipError_t e = launch_exclusive_scan_u32(a.sk.counts, nk, a.sk.block_sums, s);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    hipLaunchKernelGGL(permute_kernel, grid, block, 0, s, a.sk, a.n);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, s,
                       a.sk.counts, nk, 0u);
    return hipGetLastError();
}

hipError_t launch_surrogate_check(const CheckArgs &a, float tol, uint8_t *tile_fail, int *n_fail,
                                  hipStream_t s)
{
    const unsigned nb = (unsigned)((a.n_tiles + 255) / 256);
    hipLaunchKernelGGL(clear_check_kernel, dim3(nb), dim3(256), 0, s, a.tile_err, tile_fail, n_fail,
                       a.n_tiles);
    const long long work = a.n_tiles * kCtSamples;
    hipLaunchKernelGGL(check_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(mark_kernel, dim3(nb), dim3(256), 0, s, a.tile_err, tol, tile_fail, n_fail,
                       a.n_tiles);
    return hipGetLastError();
}

hipError_t launch_advect_tiles(const AdvectArgs &a, const uint8_t *tile_fail, int ct0, int ct1,
                               long long n_tiles, hipStream_t s)
{
    hipLaunchKernelGGL(advect_tiles_kernel, dim3((unsigned)(n_tiles * 8)), dim3(256), 0, s, a,
                       tile_fail, ct0, ct1);
    return hipGetLastError();
}

hipError_t launch_advect_grid(int dim, const AdvectArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)a.g.n_blocks), block(256);
    LaunchTimer timer(dim == 2 ? "advect_grid_kernel<2>" : "advect_grid_kernel<3>", s);
    if (dim == 2)
        hipLaunchKernelGGL(advect_grid_kernel<2>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(advect_grid_kernel<3>, grid, block, 0, s, a);
    timer.stop(s);
    return hipGetLastError();
}

hipError_t launch_advect_ab(int dim, int order, const AdvectArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)a.g.n_blocks), block(256);
    if (dim == 2) {
        if (order == 2) hipLaunchKernelGGL((advect_ab_grid_kernel<2, 2>), grid, block, 0, s, a);
        else if (order == 3) hipLaunchKernelGGL((advect_ab_grid_kernel<2, 3>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((advect_ab_grid_kernel<2, 4>), grid, block, 0, s, a);
    } else {
        if (order == 2) hipLaunchKernelGGL((advect_ab_grid_kernel<3, 2>), grid, block, 0, s, a);
        else if (order == 3) hipLaunchKernelGGL((advect_ab_grid_kernel<3, 3>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((advect_ab_grid_kernel<3, 4>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_advect_aux(int dim, const AuxArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)(a.a.g.n_blocks * 2 * dim)), block(256);
    if (dim == 2) hipLaunchKernelGGL(advect_aux_kernel<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(advect_aux_kernel<3>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_advect_snap(int dim, const SnapArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)a.a.g.n_blocks), block(256);
    if (dim == 2) hipLaunchKernelGGL(advect_snap_kernel<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(advect_snap_kernel<3>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_early_advect(int dim, const EarlyAdvArgs &a, int first, int count, hipStream_t s)
{
    const long long work = (long long)count * 7;
    dim3 grid((unsigned)((work + 255) / 256)), block(256);
    if (dim == 2) hipLaunchKernelGGL(early_advect_kernel<2>, grid, block, 0, s, a, first, count);
    else hipLaunchKernelGGL(early_advect_kernel<3>, grid, block, 0, s, a, first, count);
    return hipGetLastError();
}

hipError_t launch_interleave(int dim, int S, const float *const *u, long long nodes, int f_count,
                             long long f_first, float *out, hipStream_t s)
{
    const long long n = nodes * f_count;
    hipLaunchKernelGGL(interleave_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dim, S,
                       u[0], u[1], dim == 3 ? u[2] : u[1], n, f_first * nodes, out);
    return hipGetLastError();
}

hipError_t launch_interleave_tpair(int dim, const float *const *u, const int *n, int f_count,
                                  int f_first, float *out, hipStream_t s)
{
    const long long per_pair = (long long)(n[0] + 1) * n[1] * n[2];
    const long long pairs = f_count - 1;
    if (per_pair <= 0 || pairs <= 0) return hipSuccess;
    if (per_pair >= (1LL << 32)) return hipErrorInvalidValue;
    const unsigned bx = (unsigned)((per_pair + 255) / 256);
    const long long runs = (pairs + kTPairRun - 1) / kTPairRun;
    for (long long r0 = 0; r0 < runs; r0 += 65535) {   // grid y covers up to 65535 runs
        const unsigned by = (unsigned)(runs - r0 < 65535 ? runs - r0 : 65535);
        if (dim == 2)
            hipLaunchKernelGGL(interleave_tpair_kernel<2>, dim3(bx, by), dim3(256), 0, s, u[0], u[1],
                               u[1], n[0], n[1], 1, (long long)f_first, r0 * kTPairRun, pairs, out);
        else
            hipLaunchKernelGGL(interleave_tpair_kernel<3>, dim3(bx, by), dim3(256), 0, s, u[0], u[1],
                               u[2], n[0], n[1], n[2], (long long)f_first, r0 * kTPairRun, pairs, out);
    }
    return hipGetLastError();
}

hipError_t launch_reset_counter(int *counter, hipStream_t s)
{
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(kBatchCounters), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_advect_batched(int dim, const BatchArgs &a, int grid_blocks, hipStream_t s)
{
    dim3 grid((unsigned)grid_blocks), block(256);
    if (dim == 2)
        hipLaunchKernelGGL(advect_batched_kernel<2>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(advect_batched_kernel<3>, grid, block, 0, s, a);
    return hipGetLastError();
}

int batched_blocks_per_cu(int dim)
{
    int nb = 0;
    hipError_t e = (dim == 2)
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, advect_batched_kernel<2>, 256, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, advect_batched_kernel<3>, 256, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_advect_points(int dim, const AdvectArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)((a.ns + 255) / 256)), block(256);
    if (dim == 2)
        hipLaunchKernelGGL(advect_points_kernel<2>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(advect_points_kernel<3>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace lcs
