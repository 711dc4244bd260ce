// device_common.h -- device helpers shared by the advection kernels of the
// structured-grid and the unstructured-mesh paths: two-float arithmetic for
// positions and step sizes, the RK4 stage-point update, and the launch-order
// mapping of seed tiles (Morton curve, XCD-aware block remap).
#pragma once

#include "lcs_internal.h"

namespace lcs {

// Error-free sum: s + e == a + b exactly (Knuth's TwoSum).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

template <int D>
__device__ __forceinline__ bool finite_vec(const float *k)
{
    bool ok = true;
#pragma unroll
    for (int a = 0; a < D; ++a) ok = ok && isfinite(k[a]);
    return ok;
}

// Step-size constants as two-floats, so that the FP32 rounding of dt does not
// bias every step the same way.
struct StepConsts {
    float hh, hl;   // dt/2
    float fh, fl;   // dt
    float sh, sl;   // dt/6
};

__device__ __forceinline__ StepConsts step_consts(double dt)
{
    StepConsts c;
    c.hh = (float)(0.5 * dt); c.hl = (float)(0.5 * dt - (double)c.hh);
    c.fh = (float)dt;         c.fl = (float)(dt - (double)c.fh);
    c.sh = (float)(dt / 6.0); c.sl = (float)(dt / 6.0 - (double)c.sh);
    return c;
}

// Stage point (ph + pl) = (xh + xl) + (ch + cl) k, renormalised.
template <int D>
__device__ __forceinline__ void stage_point(const float *xh, const float *xl, float ch, float cl,
                                            const float *k, float *ph, float *pl)
{
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const float inc = fmaf(ch, k[a], cl * k[a]);
        two_sum(xh[a], xl[a] + inc, ph[a], pl[a]);
    }
}

// XCD-aware block order: workgroups are dealt round-robin to the 8 XCDs, so
// block b runs on XCD b % 8.  Give each XCD a contiguous run of the curve:
// XCDs < r take q+1 consecutive positions, the others q (q, r = divmod(B, 8)).
__device__ __forceinline__ int xcd_remap(int b, int nblocks)
{
    constexpr int kXcd = 8;
    const int q = nblocks / kXcd, r = nblocks % kXcd;
    const int x = b % kXcd, local = b / kXcd;
    return (x < r) ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

// Seed of this lane for Morton tile index m, or -1 if the tile or the lane
// falls outside the seed grid.  Morton decode with per-axis bit counts (an
// axis that runs out of bits drops out of the interleave); within the tile,
// waves and lanes are laid out as wg x wt seeds.
template <int D>
__device__ __forceinline__ long long seed_of(const SeedTiling &g, int m, int t, int *sc)
{
    int tc[3] = {0, 0, 0};
    int pos = 0;
    for (int l = 0; l < g.max_bits; ++l)
#pragma unroll
        for (int a = 0; a < D; ++a)
            if (l < g.bits[a]) tc[a] |= ((m >> (pos++)) & 1) << l;
#pragma unroll
    for (int a = 0; a < D; ++a)
        if (tc[a] >= g.ntiles[a]) return -1;
    const int w = t / kWave, l = t % kWave;
    int wc[3], lc[3];
    wc[0] = w % g.wg[0];
    wc[1] = (w / g.wg[0]) % g.wg[1];
    wc[2] = w / (g.wg[0] * g.wg[1]);
    lc[0] = l % g.wt[0];
    lc[1] = (l / g.wt[0]) % g.wt[1];
    lc[2] = l / (g.wt[0] * g.wt[1]);
    sc[0] = sc[1] = sc[2] = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        sc[a] = (tc[a] * g.wg[a] + wc[a]) * g.wt[a] + lc[a];
        if (sc[a] >= g.sn[a]) return -1;
    }
    return (long long)sc[0] + (long long)g.sn[0] * ((long long)sc[1] +
           (long long)g.sn[1] * (long long)sc[2]);
}

}  // namespace lcs
