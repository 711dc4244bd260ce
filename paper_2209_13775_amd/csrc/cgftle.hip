// cgftle.hip -- flow-map gradient, Cauchy-Green tensor, lambda_max and FTLE
// on gfx950, all in FP64 (Eq. 1; Sec. 2 Cauchy-Green filter).
//
// Launch shape: one wavefront covers 64 consecutive seeds of one x-row, a
// workgroup 4 rows.  The x-neighbours of a seed are taken from the adjacent
// lanes by cross-lane shuffles; only the two lanes at the ends of a row
// segment (and seam/edge cases) read their x-neighbour from memory.  The y-
// and z-neighbours are coalesced row reads of the FP32 positions.

#include <stdio.h>

#include "lcs_internal.h"

namespace lcs {
namespace {

constexpr int kRows = 4;   // rows (waves) per workgroup

// lambda_max of a symmetric 2x2 [[a, b], [b, c]].
__device__ __forceinline__ double lam_max2(double a, double b, double c)
{
    return 0.5 * (a + c) + hypot(0.5 * (a - c), b);
}

// Largest eigenvalue of a symmetric 3x3 by cyclic Jacobi rotations acting on
// the six distinct entries: each rotation in the (p,q) plane with
// t = tan(theta) the smaller root of t^2 + 2 tau t - 1 = 0,
// tau = (a_qq - a_pp) / (2 a_pq), zeroes a_pq; then a_pp -= t a_pq,
// a_qq += t a_pq and the third row/column turns by (c, s).
__device__ double lam_max3_jacobi(double a00, double a01, double a02, double a11, double a12,
                                  double a22)
{
    for (int sweep = 0; sweep < 32; ++sweep) {
        const double off = a01 * a01 + a02 * a02 + a12 * a12;
        const double dia = a00 * a00 + a11 * a11 + a22 * a22;
        if (!(off > 1e-36 * dia)) break;
        // (0,1) plane, third index 2
        if (a01 != 0.0) {
            const double tau = (a11 - a00) / (2.0 * a01);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
            const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
            a00 -= t * a01; a11 += t * a01; a01 = 0.0;
            const double r0 = a02, r1 = a12;
            a02 = c * r0 - s * r1; a12 = s * r0 + c * r1;
        }
        // (0,2) plane, third index 1
        if (a02 != 0.0) {
            const double tau = (a22 - a00) / (2.0 * a02);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
            const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
            a00 -= t * a02; a22 += t * a02; a02 = 0.0;
            const double r0 = a01, r2 = a12;
            a01 = c * r0 - s * r2; a12 = s * r0 + c * r2;
        }
        // (1,2) plane, third index 0
        if (a12 != 0.0) {
            const double tau = (a22 - a11) / (2.0 * a12);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + hypot(1.0, tau));
            const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
            a11 -= t * a12; a22 += t * a12; a12 = 0.0;
            const double r1 = a01, r2 = a02;
            a01 = c * r1 - s * r2; a02 = s * r1 + c * r2;
        }
    }
    return fmax(a00, fmax(a11, a22));
}

// lambda_max of a symmetric 3x3 from the trigonometric solution of its
// characteristic cubic: with q = tr/3, p = sqrt(|C - qI|_F^2 / 6) and
// B = (C - qI)/p, the eigenvalues are q + 2p cos(phi + 2 pi k/3),
// phi = acos(det(B)/2)/3; the largest is k = 0.  Near det(B)/2 = -1 (the two
// largest eigenvalues almost equal) acos is ill-conditioned, and the Jacobi
// iteration takes over.
__device__ __forceinline__ double lam_max3(double c00, double c01, double c02, double c11,
                                           double c12, double c22)
{
    const double p1 = c01 * c01 + c02 * c02 + c12 * c12;
    const double q = (c00 + c11 + c22) / 3.0;
    const double d0 = c00 - q, d1 = c11 - q, d2 = c22 - q;
    const double p2 = d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * p1;
    if (!(p2 > 0.0)) return q;   // C = qI (or NaN input: q carries it)
    const double p = sqrt(p2 / 6.0);
    const double ip = 1.0 / p;
    const double b00 = d0 * ip, b11 = d1 * ip, b22 = d2 * ip;
    const double b01 = c01 * ip, b02 = c02 * ip, b12 = c12 * ip;
    const double det = b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) +
                       b02 * (b01 * b12 - b11 * b02);
    const double r = fmin(fmax(0.5 * det, -1.0), 1.0);
    if (r < -0.999) return lam_max3_jacobi(c00, c01, c02, c11, c12, c22);
    const double phi = acos(r) / 3.0;
    return q + 2.0 * p * cos(phi);
}

__device__ __forceinline__ double ftle_of(double lam, double inv_two_T)
{
    return lam > 0.0 ? log(lam) * inv_two_T : -INFINITY;
}

// Neighbour index along an axis and the period shift of its position: wraps
// on periodic axes (shift +/- L across the seam), clamps on the others.
__device__ __forceinline__ int nbr(int i, int dir, int n, bool per, double L, double &shift)
{
    int j = i + dir;
    shift = 0.0;
    if (per) {
        if (j < 0) { j += n; shift = -L; }
        if (j >= n) { j -= n; shift = L; }
    } else {
        j = min(max(j, 0), n - 1);
    }
    return j;
}

// Flow-map gradient from auxiliary points: one thread per seed,
//   J[a][b] = (F_a(x0 + delta_b e_b) - F_a(x0 - delta_b e_b)) / (2 delta_b),
// with each final position hi + lo summed exactly in FP64; C = J^T J packed.
// No contraction, so identical positions give the oracle's C bit for bit.
template <int D>
__global__ __launch_bounds__(256) void cg_aux_kernel(CgAuxArgs A)
{
#pragma clang fp contract(off)
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.ns) return;
    const long long ns = A.ns;
    double J[3][3];
    uint8_t bad = 0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        const int qm = 2 * b, qp = 2 * b + 1;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const long long im = ((long long)a * 2 * D + qm) * ns + p;
            const long long ip = ((long long)a * 2 * D + qp) * ns + p;
            const double xm = (double)A.xa_hi[im] + (double)A.xa_lo[im];
            const double xp = (double)A.xa_hi[ip] + (double)A.xa_lo[ip];
            J[a][b] = (xp - xm) / (2.0 * A.delta[b]);
        }
        if (A.flags && (A.flags[(long long)qm * ns + p] || A.flags[(long long)qp * ns + p])) bad = 1;
    }
    int k = 0;
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
        for (int c = r; c < D; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) acc += J[a][r] * J[a][c];
            A.C[(long long)(k++) * ns + p] = acc;
        }
    if (A.sflags) A.sflags[p] = bad ? (uint8_t)LCS_FLAG_STENCIL_OUT : (uint8_t)0;
}

template <int D, bool FUSED>
__global__ __launch_bounds__(256) void cg_kernel(CgArgs A)
{
#pragma clang fp contract(off)
    const int lane = threadIdx.x % kWave;
    const int row = threadIdx.x / kWave;
    const int i = blockIdx.x * kWave + lane;
    const int j = blockIdx.y * kRows + row;
    const int k = blockIdx.z;
    const int n0 = A.n[0], n1 = A.n[1];
    const bool active = (i < n0) && (j < n1);
    const int ic = active ? i : 0;
    const long long s = (long long)ic + (long long)n0 * ((long long)(active ? j : 0) +
                        (long long)n1 * k);
    const long long ns = A.ns;

    // own position (FP32 -> FP64) and flag
    double xc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < D; ++a) xc[a] = (double)A.xf[a * ns + s];
    uint32_t fl = A.flags ? A.flags[s] : 0u;

    // x-neighbours: shuffled from lanes +-1 when they hold exactly the wanted
    // seed, otherwise read from memory
    const bool per0 = A.periodic_mask & 1u;
    double sh_m, sh_p;
    const int im = nbr(ic, -1, n0, per0, A.period[0], sh_m);
    const int ip = nbr(ic, +1, n0, per0, A.period[0], sh_p);
    double xm[3][3], xp[3][3];
    uint32_t fm = 0, fp = 0;
    {
        const bool left_ok = (lane > 0) && (im == ic - 1);
        const bool right_ok = (lane < kWave - 1) && (ip == ic + 1) && (ic + 1 < n0);
        const long long sm = s + (im - ic), sp = s + (ip - ic);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const float mine = (float)xc[a];
            const float from_left = __shfl_up(mine, 1, kWave);
            const float from_right = __shfl_down(mine, 1, kWave);
            const float vm = left_ok ? from_left : A.xf[a * ns + sm];
            const float vp = right_ok ? from_right : A.xf[a * ns + sp];
            xm[0][a] = (double)vm + (a == 0 ? sh_m : 0.0);
            xp[0][a] = (double)vp + (a == 0 ? sh_p : 0.0);
        }
        if (A.flags) {
            const int fmine = (int)fl;
            const int l_f = __shfl_up(fmine, 1, kWave);
            const int r_f = __shfl_down(fmine, 1, kWave);
            fm = left_ok ? (uint32_t)l_f : A.flags[sm];
            fp = right_ok ? (uint32_t)r_f : A.flags[sp];
        }
    }
    if (!active) return;
    fl |= fm | fp;

    // y- and z-neighbours from memory
    const int jj[3] = {i, j, k};
    const long long stride[3] = {1, (long long)n0, (long long)n0 * n1};
#pragma unroll
    for (int b = 1; b < D; ++b) {
        const bool per = (A.periodic_mask >> b) & 1u;
        double shm, shp;
        const int bm = nbr(jj[b], -1, A.n[b], per, A.period[b], shm);
        const int bp = nbr(jj[b], +1, A.n[b], per, A.period[b], shp);
        const long long sm = s + (long long)(bm - jj[b]) * stride[b];
        const long long sp = s + (long long)(bp - jj[b]) * stride[b];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            xm[b][a] = (double)A.xf[a * ns + sm] + (a == b ? shm : 0.0);
            xp[b][a] = (double)A.xf[a * ns + sp] + (a == b ? shp : 0.0);
        }
        if (A.flags) fl |= (uint32_t)A.flags[sm] | (uint32_t)A.flags[sp];
    }

    // J[a][b] = dF_a / dx_b: central differences, one-sided at non-periodic edges
    double J[3][3];
#pragma unroll
    for (int b = 0; b < D; ++b) {
        const bool per = (A.periodic_mask >> b) & 1u;
        const int ib = jj[b], nb = A.n[b];
        const double h = A.h[b];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (per || (ib > 0 && ib < nb - 1))
                J[a][b] = (xp[b][a] - xm[b][a]) / (2.0 * h);
            else if (ib == 0)
                J[a][b] = (xp[b][a] - xc[a]) / h;
            else
                J[a][b] = (xc[a] - xm[b][a]) / h;
        }
    }
    // C = J^T J, packed upper triangle
    double Cp[6];
    int q = 0;
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
        for (int c = r; c < D; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) acc += J[a][r] * J[a][c];
            Cp[q++] = acc;
        }
    if (A.sflags) A.sflags[s] = fl ? (uint8_t)LCS_FLAG_STENCIL_OUT : (uint8_t)0;
    if constexpr (!FUSED) {
#pragma unroll
        for (int r = 0; r < D * (D + 1) / 2; ++r) A.C[r * ns + s] = Cp[r];
    } else {
        double lam;
        if constexpr (D == 2)
            lam = lam_max2(Cp[0], Cp[1], Cp[2]);
        else
            lam = lam_max3(Cp[0], Cp[1], Cp[2], Cp[3], Cp[4], Cp[5]);
        if (A.lam) A.lam[s] = lam;
        if (A.ftle) A.ftle[s] = ftle_of(lam, A.inv_two_T);
    }
}

template <int D>
__global__ __launch_bounds__(256) void ftle_kernel(FtleArgs A)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    const long long n = A.n;
    double lam;
    if constexpr (D == 2)
        lam = lam_max2(A.C[p], A.C[n + p], A.C[2 * n + p]);
    else
        lam = lam_max3(A.C[p], A.C[n + p], A.C[2 * n + p], A.C[3 * n + p], A.C[4 * n + p],
                       A.C[5 * n + p]);
    if (A.lam) A.lam[p] = lam;
    if (A.ftle) A.ftle[p] = ftle_of(lam, A.inv_two_T);
}


// Eigenpairs of a symmetric dim x dim matrix (Sec. 2 Cauchy-Green filter:
// eigenvalue and eigenvector fields).  Cyclic Jacobi: each rotation zeroes
// A[p][q] (two-sided on A, one-sided on V), sweeps until the off-diagonal mass
// is negligible; then ascending order and the sign of every eigenvector fixed
// so that its largest component (the first on a tie) is positive.
template <int D>
__device__ void eig_sym(const double *c, double *ev, double (*vec)[3])
{
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    int k = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
            A[i][j] = c[k];
            A[j][i] = c[k];
            ++k;
        }
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, dia = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            dia += A[i][i] * A[i][i];
#pragma unroll
            for (int j = i + 1; j < D; ++j) off += A[i][j] * A[i][j];
        }
        if (off == 0.0 || off <= 1e-36 * dia) break;
#pragma unroll
        for (int p = 0; p < D; ++p)
#pragma unroll
            for (int q = p + 1; q < D; ++q) {
                if (A[p][q] == 0.0) continue;
                const double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (tau >= 0.0) ? 1.0 / (tau + hypot(1.0, tau))
                                              : 1.0 / (tau - hypot(1.0, tau));
                const double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
                // A <- R^T A R with R = I except R[p][p] = R[q][q] = cs, R[p][q] = sn, R[q][p] = -sn
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    const double aip = A[i][p], aiq = A[i][q];
                    A[i][p] = cs * aip - sn * aiq;
                    A[i][q] = sn * aip + cs * aiq;
                    const double vip = V[i][p], viq = V[i][q];
                    V[i][p] = cs * vip - sn * viq;
                    V[i][q] = sn * vip + cs * viq;
                }
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const double apj = A[p][j], aqj = A[q][j];
                    A[p][j] = cs * apj - sn * aqj;
                    A[q][j] = sn * apj + cs * aqj;
                }
                A[p][q] = 0.0;
                A[q][p] = 0.0;
            }
    }
    int order[3] = {0, 1, 2};
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i + 1; j < D; ++j)
            if (A[order[j]][order[j]] < A[order[i]][order[i]]) {
                const int t = order[i];
                order[i] = order[j];
                order[j] = t;
            }
#pragma unroll
    for (int e = 0; e < D; ++e) {
        const int col = order[e];
        ev[e] = A[col][col];
        int big = 0;
#pragma unroll
        for (int a = 1; a < D; ++a)
            if (fabs(V[a][col]) > fabs(V[big][col])) big = a;
        const double sg = (V[big][col] < 0.0) ? -1.0 : 1.0;
#pragma unroll
        for (int a = 0; a < D; ++a) vec[e][a] = sg * V[a][col];
    }
}

template <int D>
__global__ __launch_bounds__(256) void eig_kernel(long long n, const double *C, double *evals,
                                                  double *evecs)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    constexpr int NQ = D * (D + 1) / 2;
    double c[6], ev[3], vec[3][3];
#pragma unroll
    for (int q = 0; q < NQ; ++q) c[q] = C[q * n + p];
    eig_sym<D>(c, ev, vec);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (evals) evals[k * n + p] = ev[k];
        if (evecs)
#pragma unroll
            for (int a = 0; a < D; ++a) evecs[(k * D + a) * n + p] = vec[k][a];
    }
}

// ---- early Cauchy-Green evaluation ----------------------------------------

// Neighbour of seed coordinate c along axis b in direction dir: the wrapped
// index on a periodic axis, -1 past a non-periodic edge.
__device__ __forceinline__ int nb_index(const EarlyArgs &A, int b, int c, int dir)
{
    const int n = A.n[b];
    int j = c + dir;
    if ((A.periodic_mask >> b) & 1u) return (j + n) % n;
    return (j < 0 || j >= n) ? -1 : j;
}

__device__ __forceinline__ long long lin(const EarlyArgs &A, const int *c)
{
    return (long long)c[0] + (long long)A.n[0] * ((long long)c[1] + (long long)A.n[1] * c[2]);
}

// Gradient of the flow map at seed c from FP64 positions of the seed (xc) and
// its lower/upper neighbours (xm[b], xp[b]): central in the interior and on
// periodic axes (seam shift by the period), one-sided at non-periodic edges;
// C = J^T J packed; returns lambda_max.
template <int D>
__device__ double grad_lam(const EarlyArgs &A, const int *c, const double *xc, const double (*xm)[3],
                           const double (*xp)[3], double *Cp)
{
#pragma clang fp contract(off)
    double J[3][3];
#pragma unroll
    for (int b = 0; b < D; ++b) {
        const int n = A.n[b];
        const double h = A.h[b];
        if ((A.periodic_mask >> b) & 1u) {
            const double L = (double)n * h;
            const double sp = (c[b] + 1 >= n) ? L : 0.0;
            const double sm = (c[b] - 1 < 0) ? -L : 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const double fp = xp[b][a] + (a == b ? sp : 0.0);
                const double fm = xm[b][a] + (a == b ? sm : 0.0);
                J[a][b] = (fp - fm) / (2.0 * h);
            }
        } else if (c[b] == 0) {
#pragma unroll
            for (int a = 0; a < D; ++a) J[a][b] = (xp[b][a] - xc[a]) / h;
        } else if (c[b] == n - 1) {
#pragma unroll
            for (int a = 0; a < D; ++a) J[a][b] = (xc[a] - xm[b][a]) / h;
        } else {
#pragma unroll
            for (int a = 0; a < D; ++a) J[a][b] = (xp[b][a] - xm[b][a]) / (2.0 * h);
        }
    }
    int k = 0;
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
        for (int q = r; q < D; ++q) {
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) acc += J[a][r] * J[a][q];
            Cp[k++] = acc;
        }
    if constexpr (D == 2) return lam_max2(Cp[0], Cp[1], Cp[2]);
    else return lam_max3(Cp[0], Cp[1], Cp[2], Cp[3], Cp[4], Cp[5]);
}

__device__ __forceinline__ void seed_coords(const EarlyArgs &A, long long s, int *c)
{
    c[0] = (int)(s % A.n[0]);
    c[1] = (int)((s / A.n[0]) % A.n[1]);
    c[2] = (int)(s / ((long long)A.n[0] * A.n[1]));
}

// Earliest exit in each seed's stencil.  Seeds whose stencil ran the whole
// interval get the ordinary FTLE from xf here; the others are listed (their
// stencil is re-advected), n_s = 0 gives NaN.
template <int D>
__global__ __launch_bounds__(256) void early_mark_kernel(EarlyArgs A)
{
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= A.ns) return;
    int c[3];
    seed_coords(A, s, c);
    int nsd = A.steps_done[s];
#pragma unroll
    for (int b = 0; b < D; ++b)
#pragma unroll
        for (int dir = -1; dir <= 1; dir += 2) {
            const int j = nb_index(A, b, c[b], dir);
            if (j < 0) continue;
            int cc[3] = {c[0], c[1], c[2]};
            cc[b] = j;
            nsd = min(nsd, A.steps_done[lin(A, cc)]);
        }
    if (A.t_eff) A.t_eff[s] = (double)nsd * A.dt;
    if (nsd >= A.nsteps) {
        double xc[3] = {0, 0, 0}, xm[3][3], xp[3][3], Cp[6];
#pragma unroll
        for (int a = 0; a < D; ++a) xc[a] = (double)A.xf[a * A.ns + s];
#pragma unroll
        for (int b = 0; b < D; ++b)
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                double *dst = side ? xp[b] : xm[b];
                const int j = nb_index(A, b, c[b], side ? 1 : -1);
                int cc[3] = {c[0], c[1], c[2]};
                if (j >= 0) cc[b] = j;
                const long long t = lin(A, cc);
#pragma unroll
                for (int a = 0; a < D; ++a) dst[a] = (double)A.xf[a * A.ns + t];
            }
        const double lam = grad_lam<D>(A, c, xc, xm, xp, Cp);
        if (A.lam) A.lam[s] = lam;
        A.ftle[s] = (lam > 0.0) ? log(lam) / (2.0 * fabs((double)A.nsteps * A.dt)) : -INFINITY;
    } else if (nsd <= 0) {
        if (A.lam) A.lam[s] = __builtin_nan("");
        A.ftle[s] = __builtin_nan("");
    } else {
        const int q = atomicAdd(A.counter, 1);
        A.list[2 * q] = (int)s;
        A.list[2 * q + 1] = nsd;
    }
}

// Gradient of the listed seeds [first, first + count) from the re-advected
// stencil positions (FP64, [entry][slot][3], slot 0 = the seed, 1 + 2b + side
// = its neighbour along b), with T = n_s dt.
template <int D>
__global__ __launch_bounds__(256) void early_cg_kernel(EarlyArgs A, int first, int count)
{
    const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= count) return;
    const long long s = A.list[2 * (first + e)];
    const int nsd = A.list[2 * (first + e) + 1];
    int c[3];
    seed_coords(A, s, c);
    const double *P = A.pos + (long long)e * 7 * 3;
    double xc[3], xm[3][3], xp[3][3], Cp[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) xc[a] = P[a];
#pragma unroll
    for (int b = 0; b < D; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            xm[b][a] = P[(1 + 2 * b) * 3 + a];
            xp[b][a] = P[(2 + 2 * b) * 3 + a];
        }
    const double lam = grad_lam<D>(A, c, xc, xm, xp, Cp);
    if (A.lam) A.lam[s] = lam;
    A.ftle[s] = (lam > 0.0) ? log(lam) / (2.0 * fabs((double)nsd * A.dt)) : -INFINITY;
}

}  // namespace

hipError_t launch_eig(int dim, long long n, const double *C, double *evals, double *evecs,
                      hipStream_t s)
{
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (dim == 2) hipLaunchKernelGGL(eig_kernel<2>, grid, block, 0, s, n, C, evals, evecs);
    else hipLaunchKernelGGL(eig_kernel<3>, grid, block, 0, s, n, C, evals, evecs);
    return hipGetLastError();
}

hipError_t launch_early_mark(const EarlyArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)((a.ns + 255) / 256)), block(256);
    if (a.dim == 2) hipLaunchKernelGGL(early_mark_kernel<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(early_mark_kernel<3>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_early_cg(const EarlyArgs &a, int first, int count, hipStream_t s)
{
    dim3 grid((unsigned)((count + 255) / 256)), block(256);
    if (a.dim == 2) hipLaunchKernelGGL(early_cg_kernel<2>, grid, block, 0, s, a, first, count);
    else hipLaunchKernelGGL(early_cg_kernel<3>, grid, block, 0, s, a, first, count);
    return hipGetLastError();
}

hipError_t launch_cg_aux(const CgAuxArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)((a.ns + 255) / 256)), block(256);
    if (a.dim == 2) hipLaunchKernelGGL(cg_aux_kernel<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(cg_aux_kernel<3>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cg(const CgArgs &a, bool fused, hipStream_t s)
{
    dim3 grid((unsigned)((a.n[0] + kWave - 1) / kWave), (unsigned)((a.n[1] + kRows - 1) / kRows),
              (unsigned)(a.dim == 3 ? a.n[2] : 1));
    dim3 block(kWave * kRows);
    char name[48];
    snprintf(name, sizeof(name), "cg_kernel<%d, %s>", a.dim, fused ? "true" : "false");
    LaunchTimer timer(name, s);
    if (a.dim == 2) {
        if (fused) hipLaunchKernelGGL((cg_kernel<2, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((cg_kernel<2, false>), grid, block, 0, s, a);
    } else {
        if (fused) hipLaunchKernelGGL((cg_kernel<3, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((cg_kernel<3, false>), grid, block, 0, s, a);
    }
    timer.stop(s);
    return hipGetLastError();
}

hipError_t launch_ftle(int dim, const FtleArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    if (dim == 2) hipLaunchKernelGGL(ftle_kernel<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(ftle_kernel<3>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace lcs
