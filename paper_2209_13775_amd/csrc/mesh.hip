// mesh.hip -- unstructured-mesh kernels for gfx950 (triangles in 2D,
// tetrahedra in 3D).
//
// Preparation (once per mesh): node-to-cell adjacency (count, scan, fill),
// face neighbours and the FP64 affine map of every cell to barycentric
// coordinates, the bounding box and a uniform grid of buckets that gives every
// point a nearby start cell.
//
// Queries and advection (Sec. 3.2): a point is located by a local search that
// starts from a cell near it -- for a tracer, the cell that held its previous
// stage point -- and walks across the face opposite the most negative
// barycentric coordinate until every coordinate is >= -eps; the velocity is
// then the barycentric blend of the cell's node values in the two frames
// that bracket t, blended linearly in time.  Node velocities are stored with
// their components together (16 bytes per node in 3D), so one load fetches a
// node of one frame.  As on structured grids the RK4 state (two-float
// position, current cell and its barycentric coordinates) stays in registers
// for the whole integration.

#include "lcs_internal.h"
#include "device_common.h"

#include <climits>

#ifndef LCS_MESH_MIN_WAVES
#define LCS_MESH_MIN_WAVES 0
#endif
#if LCS_MESH_MIN_WAVES > 0
#define LCS_MESH_BOUNDS __launch_bounds__(256, LCS_MESH_MIN_WAVES)
#else
#define LCS_MESH_BOUNDS __launch_bounds__(256)
#endif

namespace lcs {
namespace {

constexpr uint32_t kOut = LCS_FLAG_OUT;
constexpr uint32_t kNonFinite = LCS_FLAG_NONFINITE;
constexpr uint32_t kTimeOut = LCS_FLAG_TIME_OUT;
constexpr uint32_t kLost = LCS_FLAG_LOST;

// ---------------------------------------------------------------------------
// Preparation
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void mesh_degree_kernel(int dim, const int32_t *cells,
                                                          long long n_cells, long long n_nodes,
                                                          uint32_t *deg, int *err)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_cells * (dim + 1)) return;
    const int v = cells[q];
    if (v < 0 || (long long)v >= n_nodes) {
        atomicOr(err, 1);
        return;
    }
    atomicAdd(&deg[v], 1u);
}

// off[v] enters as the start of node v's cell list (exclusive scan of the
// degrees) and leaves as its end, which is the start of node v+1's.
__global__ __launch_bounds__(256) void mesh_adjacency_kernel(int dim, const int32_t *cells,
                                                             long long n_cells, long long n_nodes,
                                                             uint32_t *off, int32_t *adj)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_cells * (dim + 1)) return;
    const int v = cells[q];
    if (v < 0 || (long long)v >= n_nodes) return;
    const uint32_t p = atomicAdd(&off[v], 1u);
    adj[p] = (int32_t)(q / (dim + 1));
}

// Vertices of cell c in FP64 and the inverse of its edge matrix
// E = [v1 - v0, v2 - v0 (, v3 - v0)] (rows of E^-1 map x - v0 to
// lambda_1..lambda_D).  Returns false for a degenerate cell.
template <int D>
__device__ bool cell_affine(const double *nodes, const int32_t *cells, long long c, int *nd,
                            double (*v)[3], double (*M)[3])
{
#pragma unroll
    for (int i = 0; i <= D; ++i) {
        nd[i] = cells[c * (D + 1) + i];
#pragma unroll
        for (int a = 0; a < 3; ++a) v[i][a] = (a < D) ? nodes[(long long)nd[i] * D + a] : 0.0;
    }
    double e[3][3];
    double L2 = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double l2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            e[k][a] = v[k + 1][a] - v[0][a];
            l2 += e[k][a] * e[k][a];
        }
        L2 = fmax(L2, l2);
    }
    if constexpr (D == 2) {
        const double det = e[0][0] * e[1][1] - e[0][1] * e[1][0];
        if (!(fabs(det) > 1e-12 * L2)) return false;
        const double r = 1.0 / det;
        M[0][0] = e[1][1] * r;  M[0][1] = -e[1][0] * r;  M[0][2] = 0.0;
        M[1][0] = -e[0][1] * r; M[1][1] = e[0][0] * r;   M[1][2] = 0.0;
    } else {
        double cr[3][3];   // cr[k] = e[(k+1)%3] x e[(k+2)%3]
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double *p = e[(k + 1) % 3], *q = e[(k + 2) % 3];
            cr[k][0] = p[1] * q[2] - p[2] * q[1];
            cr[k][1] = p[2] * q[0] - p[0] * q[2];
            cr[k][2] = p[0] * q[1] - p[1] * q[0];
        }
        const double det = e[0][0] * cr[0][0] + e[0][1] * cr[0][1] + e[0][2] * cr[0][2];
        if (!(fabs(det) > 1e-12 * L2 * sqrt(L2))) return false;
        const double r = 1.0 / det;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int a = 0; a < 3; ++a) M[k][a] = cr[k][a] * r;
    }
    return true;
}

// Geometry, node ids and face neighbours of every cell.  The neighbour
// across the face opposite vertex i is the other cell in the adjacency list
// of one face node that contains every face node.
template <int D>
__global__ __launch_bounds__(256) void mesh_cells_kernel(const double *nodes, const int32_t *cells,
                                                         long long n_cells, const uint32_t *off,
                                                         const int32_t *adj, float4 *rec, int *err,
                                                         unsigned long long *n_boundary)
{
    constexpr int RS = MeshGeo<D>::RS;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    int nd[4] = {-1, -1, -1, -1};
    double v[4][3], M[3][3];
    if (!cell_affine<D>(nodes, cells, c, nd, v, M)) {
        atomicOr(err, 2);
        return;
    }
    // FP32 reference point and the FP64 offset it leaves
    float r[3];
    double cc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) r[a] = (float)v[0][a];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) s += M[k][a] * ((double)r[a] - v[0][a]);
        cc[k] = s;
    }
    float4 *g = rec + c * RS;
    if constexpr (D == 3) {
        g[0] = make_float4(r[0], r[1], r[2], (float)cc[0]);
        g[1] = make_float4((float)M[0][0], (float)M[0][1], (float)M[0][2], (float)cc[1]);
        g[2] = make_float4((float)M[1][0], (float)M[1][1], (float)M[1][2], (float)cc[2]);
        g[3] = make_float4((float)M[2][0], (float)M[2][1], (float)M[2][2], 0.0f);
    } else {
        g[0] = make_float4(r[0], r[1], (float)cc[0], (float)cc[1]);
        g[1] = make_float4((float)M[0][0], (float)M[0][1], (float)M[1][0], (float)M[1][1]);
    }
    int nb[4] = {-1, -1, -1, -1};
#pragma unroll
    for (int i = 0; i <= D; ++i) {
        int face[3];
        int k = 0;
#pragma unroll
        for (int j = 0; j <= D; ++j)
            if (j != i) face[k++] = nd[j];
        const int a = face[0];
        const uint32_t start = (a == 0) ? 0u : off[a - 1], end = off[a];
        int found = -1, count = 0;
        for (uint32_t p = start; p < end; ++p) {
            const int c2 = adj[p];
            if ((long long)c2 == c) continue;
            int hits = 0;
            for (int j = 0; j <= D; ++j) {
                const int w = cells[(long long)c2 * (D + 1) + j];
#pragma unroll
                for (int f = 0; f < D; ++f) hits += (w == face[f]);
            }
            if (hits == D) {
                found = c2;
                ++count;
            }
        }
        if (count > 1) atomicOr(err, 4);
        if (found < 0) atomicAdd(n_boundary, 1ull);
        nb[i] = found;
    }
    reinterpret_cast<int4 *>(g)[MeshGeo<D>::NBR] = make_int4(nb[0], nb[1], nb[2], nb[3]);
    reinterpret_cast<int4 *>(g)[MeshGeo<D>::CONN] = make_int4(nd[0], nd[1], nd[2], D == 3 ? nd[3] : -1);
}

// Bounding box: per-block partial min/max, then one block combines them.
__global__ __launch_bounds__(256) void mesh_bbox_partial_kernel(int dim, const double *nodes,
                                                                long long n_nodes, double *part)
{
    __shared__ double sh[6][256];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < n_nodes;
         p += (long long)gridDim.x * blockDim.x)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (a < dim) {
                const double x = nodes[p * dim + a];
                lo[a] = fmin(lo[a], x);
                hi[a] = fmax(hi[a], x);
            }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        sh[a][threadIdx.x] = lo[a];
        sh[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int a = 0; a < 3; ++a) {
                sh[a][threadIdx.x] = fmin(sh[a][threadIdx.x], sh[a][threadIdx.x + w]);
                sh[3 + a][threadIdx.x] = fmax(sh[3 + a][threadIdx.x], sh[3 + a][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(64) void mesh_bbox_final_kernel(const double *part, int n_parts,
                                                             double *out)
{
    if (threadIdx.x >= 6) return;
    const int q = threadIdx.x;
    double r = (q < 3) ? INFINITY : -INFINITY;
    for (int b = 0; b < n_parts; ++b) r = (q < 3) ? fmin(r, part[b * 6 + q]) : fmax(r, part[b * 6 + q]);
    out[q] = r;
}

// Every cell marks the buckets its bounding box meets (touch) and those whose
// centre it contains (contain); atomicMin keeps the lowest cell id, so the
// result does not depend on the order in which cells run.
template <int D>
__global__ __launch_bounds__(256) void mesh_raster_kernel(const double *nodes, const int32_t *cells,
                                                          long long n_cells, MeshLocGrid g,
                                                          int *contain, int *touch)
{
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    int nd[4];
    double v[4][3], M[3][3];
    if (!cell_affine<D>(nodes, cells, c, nd, v, M)) return;
    int b0[3] = {0, 0, 0}, b1[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < D; ++a) {
        double mn = v[0][a], mx = v[0][a];
#pragma unroll
        for (int i = 1; i <= D; ++i) {
            mn = fmin(mn, v[i][a]);
            mx = fmax(mx, v[i][a]);
        }
        const double top = (double)(g.nb[a] - 1);
        b0[a] = (int)fmin(fmax(floor((mn - g.lo[a]) / g.bs[a]), 0.0), top);
        b1[a] = (int)fmin(fmax(floor((mx - g.lo[a]) / g.bs[a]), 0.0), top);
    }
    for (int bz = b0[2]; bz <= b1[2]; ++bz)
        for (int by = b0[1]; by <= b1[1]; ++by)
            for (int bx = b0[0]; bx <= b1[0]; ++bx) {
                const long long b = bx + (long long)g.nb[0] * (by + (long long)g.nb[1] * bz);
                atomicMin(&touch[b], (int)c);
                const int bb[3] = {bx, by, bz};
                double d[3], lmin, l0 = 1.0;
#pragma unroll
                for (int a = 0; a < D; ++a) d[a] = g.lo[a] + ((double)bb[a] + 0.5) * g.bs[a] - v[0][a];
                lmin = INFINITY;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    double l = 0.0;
#pragma unroll
                    for (int a = 0; a < D; ++a) l += M[k][a] * d[a];
                    lmin = fmin(lmin, l);
                    l0 -= l;
                }
                lmin = fmin(lmin, l0);
                if (lmin >= -1e-12) atomicMin(&contain[b], (int)c);
            }
}

__global__ __launch_bounds__(256) void mesh_locator_finish_kernel(const int *contain,
                                                                  const int *touch, long long n,
                                                                  int *loc)
{
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const int c = contain[b], t = touch[b];
    loc[b] = (c != INT_MAX) ? c : ((t != INT_MAX) ? t : -1);
}

// ---------------------------------------------------------------------------
// Location and interpolation
// ---------------------------------------------------------------------------

// Barycentric coordinates of the two-float point (ph + pl) in the cell whose
// geometry is q.  x - r is formed from the two-float point and the FP32
// reference point, so it is accurate to FP32 rounding of the difference.
template <int D>
__device__ __forceinline__ void barycentric(const float4 *q, const float *ph, const float *pl,
                                            float *lam)
{
    if constexpr (D == 3) {
        const float d0 = (ph[0] - q[0].x) + pl[0];
        const float d1 = (ph[1] - q[0].y) + pl[1];
        const float d2 = (ph[2] - q[0].z) + pl[2];
        lam[1] = fmaf(q[1].x, d0, fmaf(q[1].y, d1, fmaf(q[1].z, d2, q[0].w)));
        lam[2] = fmaf(q[2].x, d0, fmaf(q[2].y, d1, fmaf(q[2].z, d2, q[1].w)));
        lam[3] = fmaf(q[3].x, d0, fmaf(q[3].y, d1, fmaf(q[3].z, d2, q[2].w)));
        lam[0] = 1.0f - (lam[1] + lam[2] + lam[3]);
    } else {
        const float d0 = (ph[0] - q[0].x) + pl[0];
        const float d1 = (ph[1] - q[0].y) + pl[1];
        lam[1] = fmaf(q[1].x, d0, fmaf(q[1].y, d1, q[0].z));
        lam[2] = fmaf(q[1].z, d0, fmaf(q[1].w, d1, q[0].w));
        lam[0] = 1.0f - (lam[1] + lam[2]);
    }
}

#ifndef LCS_MESH_CACHE
#define LCS_MESH_CACHE 1
#endif

// Per-tracer copies, in registers, of the geometry of the cell visited last
// and of the node values of the cell and frame pair sampled last.  RK4 stage
// points and successive steps mostly stay in one cell, and then the loads are
// skipped; the values are the same either way.
template <int D>
struct MeshCache {
    int gcell = -1;                  // cell whose geometry is in q (-1: none)
    float4 q[MeshGeo<D>::G];
    int vcell = -1;                  // cell whose node values are in ua/ub (-1: none)
    long long vbase = -1;            // frame base of those values
    float ua[D + 1][D], ub[D + 1][D];   // [node][component], frames f and f+1
};

// Local cell search from cell c (updated in place).  Returns 0 with lam set
// when the point is in c (every coordinate >= -eps), kOut when the walk
// reaches a boundary face, kLost after max_walk steps.  The point must be
// finite.
template <int D>
__device__ __forceinline__ uint32_t walk(const MeshDev &m, const float *ph, const float *pl, int &c,
                                         float *lam, MeshCache<D> &mc)
{
    constexpr int G = MeshGeo<D>::G;
    for (int s = 0; s < m.max_walk; ++s) {
        if (!LCS_MESH_CACHE || c != mc.gcell) {
            const float4 *g = m.rec + (long long)c * MeshGeo<D>::RS;
#pragma unroll
            for (int i = 0; i < G; ++i) mc.q[i] = g[i];
            mc.gcell = c;
        }
        barycentric<D>(mc.q, ph, pl, lam);
        float lmin = lam[0];
        int imin = 0;
#pragma unroll
        for (int i = 1; i <= D; ++i)
            if (lam[i] < lmin) {
                lmin = lam[i];
                imin = i;
            }
        if (lmin >= -m.eps) return 0;
        const int4 nb = reinterpret_cast<const int4 *>(m.rec + (long long)c * MeshGeo<D>::RS)[MeshGeo<D>::NBR];
        const int next = (imin == 0) ? nb.x : (imin == 1) ? nb.y : (imin == 2) ? nb.z : nb.w;
        if (next < 0) return kOut;
        c = next;
    }
    return kLost;
}

// First location of a point: start cell from its bucket, then the walk.
template <int D>
__device__ __forceinline__ uint32_t first_locate(const MeshDev &m, const float *ph, const float *pl,
                                                 int &c, float *lam, MeshCache<D> &mc)
{
    long long b = 0, stride = 1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const float top = (float)(m.nb[a] - 1);
        const float f = fminf(fmaxf(floorf((ph[a] - m.lo[a]) * m.inv_bs[a]), 0.0f), top);
        b += (long long)f * stride;
        stride *= m.nb[a];
    }
    c = m.loc[b];
    if (c < 0) return kOut;
    return walk<D>(m, ph, pl, c, lam, mc);
}

__device__ __forceinline__ void mesh_frame_at(const MeshFramesDev &f, double t, long long &base,
                                              float &alpha)
{
    double tau = (t - f.t_first) * f.inv_dt_frame;
    tau = fmin(fmax(tau, 0.0), (double)(f.n_frames - 1));
    const int fi = min((int)floor(tau), f.n_frames - 2);
    alpha = (float)(tau - (double)fi);
    base = (long long)fi * f.frame_stride;
}

__device__ __forceinline__ void mesh_frame_at_uniform(const MeshFramesDev &f, double t,
                                                      long long &base, float &alpha)
{
    double tau = (t - f.t_first) * f.inv_dt_frame;
    tau = fmin(fmax(tau, 0.0), (double)(f.n_frames - 1));
    const int fi = __builtin_amdgcn_readfirstlane(min((int)floor(tau), f.n_frames - 2));
    alpha = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint((float)(tau - (double)fi))));
    base = (long long)fi * f.frame_stride;
}

// Node record of one frame: 16 bytes (3D) or 8 bytes (2D) at a 32-bit byte
// offset from the frame base.
__device__ __forceinline__ float4 load_node4(const float *base, int node)
{
    return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) +
                                             (uint32_t)node * 16u);
}

__device__ __forceinline__ float2 load_node2(const float *base, int node)
{
    return *reinterpret_cast<const float2 *>(reinterpret_cast<const char *>(base) +
                                             (uint32_t)node * 8u);
}

// u = (1 - alpha) sum_i lam_i u_f(node_i) + alpha sum_i lam_i u_{f+1}(node_i)
template <int D>
__device__ __forceinline__ void mesh_velocity(const MeshDev &m, const MeshFramesDev &f, int c,
                                              const float *lam, long long base, float alpha,
                                              float *out, MeshCache<D> &mc)
{
#pragma clang fp contract(off)
    if (!LCS_MESH_CACHE || c != mc.vcell || base != mc.vbase) {
        const int4 cn = reinterpret_cast<const int4 *>(m.rec + (long long)c * MeshGeo<D>::RS)[MeshGeo<D>::CONN];
        const int nd[4] = {cn.x, cn.y, cn.z, cn.w};
        const float *A = f.u + base;
        const float *B = A + f.frame_stride;
#pragma unroll
        for (int i = 0; i <= D; ++i) {
            if constexpr (D == 3) {
                const float4 va = load_node4(A, nd[i]), vb = load_node4(B, nd[i]);
                mc.ua[i][0] = va.x; mc.ua[i][1] = va.y; mc.ua[i][2] = va.z;
                mc.ub[i][0] = vb.x; mc.ub[i][1] = vb.y; mc.ub[i][2] = vb.z;
            } else {
                const float2 va = load_node2(A, nd[i]), vb = load_node2(B, nd[i]);
                mc.ua[i][0] = va.x; mc.ua[i][1] = va.y;
                mc.ub[i][0] = vb.x; mc.ub[i][1] = vb.y;
            }
        }
        mc.vcell = c;
        mc.vbase = base;
    }
    float ua[3] = {0.0f, 0.0f, 0.0f}, ub[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i <= D; ++i)
#pragma unroll
        for (int k = 0; k < D; ++k) {
            ua[k] = fmaf(lam[i], mc.ua[i][k], ua[k]);
            ub[k] = fmaf(lam[i], mc.ub[i][k], ub[k]);
        }
    const float a1 = alpha, a0 = 1.0f - alpha;
#pragma unroll
    for (int k = 0; k < D; ++k) out[k] = fmaf(a1, ub[k], a0 * ua[k]);
}

// Stage point: finite, then located by a walk from cell c (updated).
template <int D>
__device__ __forceinline__ uint32_t stage_locate(const MeshDev &m, const float *ph, const float *pl,
                                                 int &c, float *lam, MeshCache<D> &mc)
{
    if (!finite_vec<D>(ph)) return kNonFinite;
    return walk<D>(m, ph, pl, c, lam, mc);
}

// Classical RK4 on the mesh field for steps 0 <= n < nsteps from t0, the
// tracer state (two-float position, its cell c and barycentric coordinates
// lam) updated in place.  Same exit reading as on structured grids: a stage
// point or new position that is non-finite or outside the mesh (or a search
// past its step limit, or a non-finite velocity) rejects the step and
// freezes the tracer.
template <int D, bool UNIFORM_T>
__device__ uint32_t mesh_advect_steps(const MeshDev &m, const MeshFramesDev &f, float *xh,
                                      float *xl, int &c, float *lam, double t0, double dt,
                                      int nsteps, MeshCache<D> &mc)
{
    uint32_t fl = 0;
    const StepConsts sc = step_consts(dt);
    for (int n = 0; n < nsteps; ++n) {
        const double t = t0 + (double)n * dt;
        long long b1, b2, b4;
        float al1, al2, al4;
        if constexpr (UNIFORM_T) {
            mesh_frame_at_uniform(f, t, b1, al1);
            mesh_frame_at_uniform(f, t + 0.5 * dt, b2, al2);
            mesh_frame_at_uniform(f, t + dt, b4, al4);
        } else {
            mesh_frame_at(f, t, b1, al1);
            mesh_frame_at(f, t + 0.5 * dt, b2, al2);
            mesh_frame_at(f, t + dt, b4, al4);
        }
        float k1[3], k2[3], k3[3], k4[3], ph[3], pl[3], ls[4];
        int cs = c;

        mesh_velocity<D>(m, f, c, lam, b1, al1, k1, mc);
        if (!finite_vec<D>(k1)) { fl = kNonFinite; break; }
        stage_point<D>(xh, xl, sc.hh, sc.hl, k1, ph, pl);
        if ((fl = stage_locate<D>(m, ph, pl, cs, ls, mc))) break;

        mesh_velocity<D>(m, f, cs, ls, b2, al2, k2, mc);
        if (!finite_vec<D>(k2)) { fl = kNonFinite; break; }
        stage_point<D>(xh, xl, sc.hh, sc.hl, k2, ph, pl);
        if ((fl = stage_locate<D>(m, ph, pl, cs, ls, mc))) break;

        mesh_velocity<D>(m, f, cs, ls, b2, al2, k3, mc);
        if (!finite_vec<D>(k3)) { fl = kNonFinite; break; }
        stage_point<D>(xh, xl, sc.fh, sc.fl, k3, ph, pl);
        if ((fl = stage_locate<D>(m, ph, pl, cs, ls, mc))) break;

        mesh_velocity<D>(m, f, cs, ls, b4, al4, k4, mc);
        if (!finite_vec<D>(k4)) { fl = kNonFinite; break; }

        float nh[3], nl[3];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const float sum = (k1[a] + k4[a]) + 2.0f * (k2[a] + k3[a]);
            const float inc = fmaf(sc.sh, sum, sc.sl * sum);
            two_sum(xh[a], xl[a] + inc, nh[a], nl[a]);
        }
        if ((fl = stage_locate<D>(m, nh, nl, cs, ls, mc))) break;
#pragma unroll
        for (int a = 0; a < D; ++a) { xh[a] = nh[a]; xl[a] = nl[a]; }
        c = cs;
#pragma unroll
        for (int i = 0; i <= D; ++i) lam[i] = ls[i];
    }
    return fl;
}

template <int D>
__global__ LCS_MESH_BOUNDS void mesh_advect_grid_kernel(MeshAdvectArgs A)
{
    const int mi = xcd_remap((int)blockIdx.x, A.g.n_blocks);
    int sc[3];
    const long long s = seed_of<D>(A.g, mi, threadIdx.x, sc);
    if (s < 0) return;
    float xh[3], xl[3], lam[4];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double x0 = A.g.s_origin[a] + (double)sc[a] * A.g.s_spacing[a];
        xh[a] = (float)x0;
        xl[a] = (float)(x0 - (double)xh[a]);
    }
    int c = -1;
    MeshCache<D> mc;
    uint32_t fl = first_locate<D>(A.m, xh, xl, c, lam, mc);
    const bool located = (fl == 0);
    if (located)
        fl = mesh_advect_steps<D, true>(A.m, A.f, xh, xl, c, lam, A.t0, A.dt, A.nsteps, mc);
#pragma unroll
    for (int a = 0; a < D; ++a) A.xf[a * A.ns + s] = xh[a] + xl[a];
    if (A.cell) A.cell[s] = located ? (long long)c : -1LL;
    if (A.flags) A.flags[s] = (uint8_t)fl;
}

template <int D>
__global__ LCS_MESH_BOUNDS void mesh_advect_points_kernel(MeshAdvectArgs A)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.ns) return;
    float xh[3], xl[3] = {0.0f, 0.0f, 0.0f}, lam[4];
#pragma unroll
    for (int a = 0; a < D; ++a) xh[a] = A.x0[a * A.ns + p];
    const double t0 = A.t0v[p];
    const double t1 = t0 + A.T;
    uint32_t fl;
    int c = -1;
    MeshCache<D> mc;
    bool located = false;
    if (!(t0 >= A.f.t_first && t0 <= A.f.t_last && t1 >= A.f.t_first && t1 <= A.f.t_last)) {
        fl = kTimeOut;
    } else if (!finite_vec<D>(xh)) {
        fl = kNonFinite;
    } else {
        fl = first_locate<D>(A.m, xh, xl, c, lam, mc);
        located = (fl == 0);
        if (located)
            fl = mesh_advect_steps<D, false>(A.m, A.f, xh, xl, c, lam, t0, A.dt, A.nsteps,
                                             mc);
    }
#pragma unroll
    for (int a = 0; a < D; ++a) A.xf[a * A.ns + p] = xh[a] + xl[a];
    if (A.cell) A.cell[p] = located ? (long long)c : -1LL;
    if (A.flags) A.flags[p] = (uint8_t)fl;
}

template <int D>
__global__ __launch_bounds__(256) void mesh_locate_kernel(MeshDev m, const float *x, long long n,
                                                          long long *cell, float *lam_out)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float xh[3], xl[3] = {0.0f, 0.0f, 0.0f}, lam[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int a = 0; a < D; ++a) xh[a] = x[a * n + p];
    int c = -1;
    MeshCache<D> mc;
    long long r = -1;
    if (finite_vec<D>(xh)) {
        const uint32_t fl = first_locate<D>(m, xh, xl, c, lam, mc);
        r = (fl == 0) ? (long long)c : (fl == kLost ? -2LL : -1LL);
    }
    cell[p] = r;
    if (lam_out)
#pragma unroll
        for (int i = 0; i <= D; ++i) lam_out[i * n + p] = lam[i];
}

template <int D>
__global__ __launch_bounds__(256) void mesh_velocity_kernel(MeshDev m, MeshFramesDev f,
                                                            const float *x, const double *t,
                                                            long long n, float *u, long long *cell)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float xh[3], xl[3] = {0.0f, 0.0f, 0.0f}, lam[4], out[3];
#pragma unroll
    for (int a = 0; a < D; ++a) xh[a] = x[a * n + p];
    int c = -1;
    MeshCache<D> mc;
    long long r = -1;
    bool ok = false;
    if (finite_vec<D>(xh)) {
        const uint32_t fl = first_locate<D>(m, xh, xl, c, lam, mc);
        ok = (fl == 0);
        r = ok ? (long long)c : (fl == kLost ? -2LL : -1LL);
    }
    if (ok) {
        long long base;
        float alpha;
        mesh_frame_at(f, t[p], base, alpha);
        mesh_velocity<D>(m, f, c, lam, base, alpha, out, mc);
    } else {
#pragma unroll
        for (int a = 0; a < D; ++a) out[a] = __builtin_nanf("");
    }
#pragma unroll
    for (int a = 0; a < D; ++a) u[a * n + p] = out[a];
    if (cell) cell[p] = r;
}

unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_mesh_degree(int dim, const int32_t *cells, long long n_cells, long long n_nodes,
                              uint32_t *deg, int *err, hipStream_t s)
{
    hipLaunchKernelGGL(mesh_degree_kernel, dim3(blocks_for(n_cells * (dim + 1))), dim3(256), 0, s,
                       dim, cells, n_cells, n_nodes, deg, err);
    return hipGetLastError();
}

hipError_t launch_mesh_adjacency(int dim, const int32_t *cells, long long n_cells,
                                 long long n_nodes, uint32_t *off, int32_t *adj, hipStream_t s)
{
    hipLaunchKernelGGL(mesh_adjacency_kernel, dim3(blocks_for(n_cells * (dim + 1))), dim3(256), 0,
                       s, dim, cells, n_cells, n_nodes, off, adj);
    return hipGetLastError();
}

hipError_t launch_mesh_cells(int dim, const double *nodes, const int32_t *cells, long long n_cells,
                             const uint32_t *off, const int32_t *adj, float4 *rec, int *err,
                             unsigned long long *n_boundary, hipStream_t s)
{
    if (dim == 2)
        hipLaunchKernelGGL(mesh_cells_kernel<2>, dim3(blocks_for(n_cells)), dim3(256), 0, s, nodes,
                           cells, n_cells, off, adj, rec, err, n_boundary);
    else
        hipLaunchKernelGGL(mesh_cells_kernel<3>, dim3(blocks_for(n_cells)), dim3(256), 0, s, nodes,
                           cells, n_cells, off, adj, rec, err, n_boundary);
    return hipGetLastError();
}

hipError_t launch_mesh_bbox(int dim, const double *nodes, long long n_nodes, double *part,
                            int n_parts, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(mesh_bbox_partial_kernel, dim3((unsigned)n_parts), dim3(256), 0, s, dim,
                       nodes, n_nodes, part);
    hipLaunchKernelGGL(mesh_bbox_final_kernel, dim3(1), dim3(64), 0, s, part, n_parts, out);
    return hipGetLastError();
}

hipError_t launch_mesh_raster(int dim, const double *nodes, const int32_t *cells, long long n_cells,
                              const MeshLocGrid &g, int *contain, int *touch, hipStream_t s)
{
    if (dim == 2)
        hipLaunchKernelGGL(mesh_raster_kernel<2>, dim3(blocks_for(n_cells)), dim3(256), 0, s, nodes,
                           cells, n_cells, g, contain, touch);
    else
        hipLaunchKernelGGL(mesh_raster_kernel<3>, dim3(blocks_for(n_cells)), dim3(256), 0, s, nodes,
                           cells, n_cells, g, contain, touch);
    return hipGetLastError();
}

hipError_t launch_mesh_locator_finish(const int *contain, const int *touch, long long n, int *loc,
                                      hipStream_t s)
{
    hipLaunchKernelGGL(mesh_locator_finish_kernel, dim3(blocks_for(n)), dim3(256), 0, s, contain,
                       touch, n, loc);
    return hipGetLastError();
}

hipError_t launch_mesh_locate(int dim, const MeshDev &m, const float *x, long long n,
                              long long *cell, float *lam, hipStream_t s)
{
    if (dim == 2)
        hipLaunchKernelGGL(mesh_locate_kernel<2>, dim3(blocks_for(n)), dim3(256), 0, s, m, x, n,
                           cell, lam);
    else
        hipLaunchKernelGGL(mesh_locate_kernel<3>, dim3(blocks_for(n)), dim3(256), 0, s, m, x, n,
                           cell, lam);
    return hipGetLastError();
}

hipError_t launch_mesh_velocity(int dim, const MeshDev &m, const MeshFramesDev &f, const float *x,
                                const double *t, long long n, float *u, long long *cell,
                                hipStream_t s)
{
    if (dim == 2)
        hipLaunchKernelGGL(mesh_velocity_kernel<2>, dim3(blocks_for(n)), dim3(256), 0, s, m, f, x,
                           t, n, u, cell);
    else
        hipLaunchKernelGGL(mesh_velocity_kernel<3>, dim3(blocks_for(n)), dim3(256), 0, s, m, f, x,
                           t, n, u, cell);
    return hipGetLastError();
}

hipError_t launch_mesh_advect(int dim, const MeshAdvectArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)a.g.n_blocks), block(256);
    if (dim == 2) hipLaunchKernelGGL(mesh_advect_grid_kernel<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(mesh_advect_grid_kernel<3>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mesh_advect_points(int dim, const MeshAdvectArgs &a, hipStream_t s)
{
    dim3 grid(blocks_for(a.ns)), block(256);
    if (dim == 2) hipLaunchKernelGGL(mesh_advect_points_kernel<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(mesh_advect_points_kernel<3>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace lcs
