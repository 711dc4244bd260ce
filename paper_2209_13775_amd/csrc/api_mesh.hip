// api_mesh.hip -- C ABI of the unstructured-mesh path: mesh object lifetime
// (device-side preparation), point location, velocity queries and RK4
// advection of seed grids and points.  Host code validates every argument
// before anything is enqueued.

#include "lcs_internal.h"

#include <climits>
#include <cmath>
#include <cstring>
#include <vector>

namespace {

constexpr long long kMaxMeshNodes = (1LL << 28) - 1;   // 16-byte node records, 32-bit offsets
constexpr long long kMaxMeshCells = (1LL << 30) - 1;   // (dim+1) * n_cells adjacency entries < 2^32
constexpr long long kMaxBuckets = 1LL << 24;
constexpr int kBboxParts = 256;

}  // namespace

struct lcs_mesh {
    int dim = 0;
    long long n_nodes = 0, n_cells = 0;
    int device = -1;
    float4 *rec = nullptr;   // [n_cells][RS] geometry, neighbours, node ids
    int *loc = nullptr;
    int nb[3] = {1, 1, 1};
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, bs[3] = {1, 1, 1};
    long long n_boundary = 0;
    long long bytes = 0;
};

namespace {

void free_mesh(lcs_mesh *m)
{
    if (!m) return;
    if (m->rec) (void)hipFree(m->rec);
    if (m->loc) (void)hipFree(m->loc);
    delete m;
}

// Device buffers that live only while a mesh is being built.
struct Scratch {
    std::vector<void *> ptrs;
    ~Scratch()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <class T>
    hipError_t alloc(T **p, size_t bytes)
    {
        hipError_t e = hipMalloc(reinterpret_cast<void **>(p), bytes < 16 ? 16 : bytes);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
};

lcs_status check_mesh(const lcs_mesh *m)
{
    if (!m) return lcs::set_error(LCS_E_ARG, "mesh is NULL (create one with lcs_mesh_create)");
    return LCS_OK;
}

lcs_status check_frames(const lcs_mesh *m, const lcs_mesh_frames_t *f)
{
    if (!f) return lcs::set_error(LCS_E_ARG, "frames descriptor is NULL");
    if (f->reserved != 0) return lcs::set_error(LCS_E_ARG, "frames reserved field must be 0");
    if (f->n_frames < 2) return lcs::set_error(LCS_E_SHAPE, "need >= 2 frames");
    if (!(std::isfinite(f->t_first) && std::isfinite(f->dt_frame) && f->dt_frame > 0.0))
        return lcs::set_error(LCS_E_ARG, "bad t_first/dt_frame");
    if (!f->u) return lcs::set_error(LCS_E_ARG, "frames u is NULL");
    const uintptr_t align = (m->dim == 3) ? 16u : 8u;
    if (reinterpret_cast<uintptr_t>(f->u) % align)
        return lcs::set_error(LCS_E_ARG, "frames u must be %d-byte aligned", (int)align);
    return LCS_OK;
}

lcs::MeshDev mesh_dev(const lcs_mesh *m)
{
    lcs::MeshDev d;
    memset(&d, 0, sizeof(d));
    d.rec = m->rec;
    d.loc = m->loc;
    for (int a = 0; a < 3; ++a) {
        d.nb[a] = m->nb[a];
        d.lo[a] = (float)m->lo[a];
        d.inv_bs[a] = (float)(1.0 / m->bs[a]);
    }
    d.eps = (float)LCS_MESH_EPS;
    d.max_walk = LCS_MESH_MAX_WALK;
    return d;
}

lcs::MeshFramesDev frames_dev(const lcs_mesh *m, const lcs_mesh_frames_t *f)
{
    lcs::MeshFramesDev d;
    memset(&d, 0, sizeof(d));
    d.u = f->u;
    d.frame_stride = m->n_nodes * (m->dim == 3 ? 4 : 2);
    d.n_frames = f->n_frames;
    d.t_first = f->t_first;
    d.inv_dt_frame = 1.0 / f->dt_frame;
    d.t_last = f->t_first + (double)(f->n_frames - 1) * f->dt_frame;
    return d;
}

// Bucket grid of about one cell per bucket over the bounding box, at most
// kMaxBuckets buckets; a flat axis gets one bucket.
void bucket_grid(lcs_mesh *m)
{
    double vol = 1.0;
    int flat = 0;
    for (int a = 0; a < m->dim; ++a) {
        const double ext = m->hi[a] - m->lo[a];
        if (ext > 0.0) vol *= ext;
        else ++flat;
    }
    const int live = m->dim - flat;
    double edge = (live > 0) ? pow(vol / (double)m->n_cells, 1.0 / live) : 1.0;
    for (;;) {
        long long total = 1;
        for (int a = 0; a < 3; ++a) {
            const double ext = (a < m->dim) ? m->hi[a] - m->lo[a] : 0.0;
            long long k = (ext > 0.0) ? (long long)ceil(ext / edge) : 1;
            if (k < 1) k = 1;
            m->nb[a] = (int)k;
            m->bs[a] = (ext > 0.0) ? ext / (double)k : 1.0;
            total *= k;
        }
        if (total <= kMaxBuckets) break;
        edge *= 1.25;
    }
}

#define MESH_HIP(call, what)                                        \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) {                                     \
            free_mesh(m);                                           \
            return lcs::hip_error(e_, what);                        \
        }                                                           \
    } while (0)

}  // namespace

extern "C" {

lcs_status lcs_mesh_create(const lcs_mesh_desc_t *desc, lcs_mesh_t *out, void *stream)
{
    if (!desc || !out) return lcs::set_error(LCS_E_ARG, "desc and out must not be NULL");
    *out = nullptr;
    if (desc->dim != 2 && desc->dim != 3) return lcs::set_error(LCS_E_ARG, "mesh dim must be 2 or 3");
    if (desc->reserved != 0) return lcs::set_error(LCS_E_ARG, "mesh reserved field must be 0");
    if (desc->n_nodes < 1 || desc->n_nodes > kMaxMeshNodes)
        return lcs::set_error(LCS_E_SHAPE, "n_nodes must be in [1, 2^28)");
    if (desc->n_cells < 1 || desc->n_cells > kMaxMeshCells)
        return lcs::set_error(LCS_E_SHAPE, "n_cells must be in [1, 2^30)");
    if (!desc->nodes || !desc->cells) return lcs::set_error(LCS_E_ARG, "nodes and cells must not be NULL");

    hipStream_t s = (hipStream_t)stream;
    const int D = desc->dim;
    const long long nn = desc->n_nodes, nc = desc->n_cells;
    lcs_mesh *m = new lcs_mesh();
    m->dim = D;
    m->n_nodes = nn;
    m->n_cells = nc;
    MESH_HIP(hipGetDevice(&m->device), "hipGetDevice");
    const int RS = (D == 3) ? lcs::MeshGeo<3>::RS : lcs::MeshGeo<2>::RS;
    MESH_HIP(hipMalloc(&m->rec, sizeof(float4) * RS * nc), "hipMalloc(cell records)");
    m->bytes = (long long)sizeof(float4) * RS * nc;

    Scratch tmp;
    uint32_t *off = nullptr, *sums = nullptr;
    int32_t *adj = nullptr;
    int *err = nullptr;
    unsigned long long *nbnd = nullptr;
    double *part = nullptr, *box = nullptr;
    const long long n_adj = nc * (D + 1);
    MESH_HIP(tmp.alloc(&off, sizeof(uint32_t) * nn), "hipMalloc(off)");
    MESH_HIP(tmp.alloc(&sums, sizeof(uint32_t) * (lcs::exclusive_scan_sums_needed(nn) + 1)),
             "hipMalloc(sums)");
    MESH_HIP(tmp.alloc(&adj, sizeof(int32_t) * n_adj), "hipMalloc(adj)");
    MESH_HIP(tmp.alloc(&err, sizeof(int)), "hipMalloc(err)");
    MESH_HIP(tmp.alloc(&nbnd, sizeof(unsigned long long)), "hipMalloc(nbnd)");
    MESH_HIP(tmp.alloc(&part, sizeof(double) * 6 * kBboxParts), "hipMalloc(part)");
    MESH_HIP(tmp.alloc(&box, sizeof(double) * 6), "hipMalloc(box)");
    MESH_HIP(hipMemsetAsync(off, 0, sizeof(uint32_t) * nn, s), "memset");
    MESH_HIP(hipMemsetAsync(err, 0, sizeof(int), s), "memset");
    MESH_HIP(hipMemsetAsync(nbnd, 0, sizeof(unsigned long long), s), "memset");

    // 1. node degrees; stop here on an invalid node id (nothing reads nodes yet)
    MESH_HIP(lcs::launch_mesh_degree(D, desc->cells, nc, nn, off, err, s), "mesh degree");
    int h_err = 0;
    MESH_HIP(hipMemcpyAsync(&h_err, err, sizeof(int), hipMemcpyDeviceToHost, s), "copy err");
    MESH_HIP(hipStreamSynchronize(s), "sync");
    if (h_err & 1) {
        free_mesh(m);
        return lcs::set_error(LCS_E_SHAPE, "a cell names a node id outside [0, n_nodes)");
    }
    // 2. adjacency lists, 3. geometry + neighbours, 4. bounding box
    MESH_HIP(lcs::launch_exclusive_scan_u32(off, nn, sums, s), "mesh scan");
    MESH_HIP(lcs::launch_mesh_adjacency(D, desc->cells, nc, nn, off, adj, s), "mesh adjacency");
    MESH_HIP(lcs::launch_mesh_cells(D, desc->nodes, desc->cells, nc, off, adj, m->rec, err, nbnd, s),
             "mesh cells");
    MESH_HIP(lcs::launch_mesh_bbox(D, desc->nodes, nn, part, kBboxParts, box, s), "mesh bbox");
    double h_box[6];
    unsigned long long h_nb = 0;
    MESH_HIP(hipMemcpyAsync(&h_err, err, sizeof(int), hipMemcpyDeviceToHost, s), "copy err");
    MESH_HIP(hipMemcpyAsync(&h_nb, nbnd, sizeof(h_nb), hipMemcpyDeviceToHost, s), "copy nbnd");
    MESH_HIP(hipMemcpyAsync(h_box, box, sizeof(h_box), hipMemcpyDeviceToHost, s), "copy box");
    MESH_HIP(hipStreamSynchronize(s), "sync");
    if (h_err & 2) {
        free_mesh(m);
        return lcs::set_error(LCS_E_SHAPE, "degenerate (zero-measure or non-finite) cell");
    }
    if (h_err & 4) {
        free_mesh(m);
        return lcs::set_error(LCS_E_SHAPE, "a face is shared by more than two cells");
    }
    for (int a = 0; a < 3; ++a) {
        m->lo[a] = (a < D) ? h_box[a] : 0.0;
        m->hi[a] = (a < D) ? h_box[3 + a] : 0.0;
    }
    m->n_boundary = (long long)h_nb;

    // 5. first-location buckets
    bucket_grid(m);
    const long long nbt = (long long)m->nb[0] * m->nb[1] * m->nb[2];
    int *contain = nullptr, *touch = nullptr;
    MESH_HIP(hipMalloc(&m->loc, sizeof(int) * nbt), "hipMalloc(loc)");
    m->bytes += (long long)sizeof(int) * nbt;
    MESH_HIP(tmp.alloc(&contain, sizeof(int) * nbt), "hipMalloc(contain)");
    MESH_HIP(tmp.alloc(&touch, sizeof(int) * nbt), "hipMalloc(touch)");
    MESH_HIP(lcs::launch_fill_u32(reinterpret_cast<uint32_t *>(contain), nbt, (uint32_t)INT_MAX, s),
             "fill");
    MESH_HIP(lcs::launch_fill_u32(reinterpret_cast<uint32_t *>(touch), nbt, (uint32_t)INT_MAX, s),
             "fill");
    lcs::MeshLocGrid lg;
    for (int a = 0; a < 3; ++a) {
        lg.lo[a] = m->lo[a];
        lg.bs[a] = m->bs[a];
        lg.nb[a] = m->nb[a];
    }
    MESH_HIP(lcs::launch_mesh_raster(D, desc->nodes, desc->cells, nc, lg, contain, touch, s),
             "mesh raster");
    MESH_HIP(lcs::launch_mesh_locator_finish(contain, touch, nbt, m->loc, s), "mesh locator");
    MESH_HIP(hipStreamSynchronize(s), "sync");
    *out = m;
    return lcs::clear_error();
}

void lcs_mesh_destroy(lcs_mesh_t mesh)
{
    if (!mesh) return;
    (void)hipDeviceSynchronize();
    free_mesh(mesh);
}

lcs_status lcs_mesh_info(lcs_mesh_t mesh, lcs_mesh_info_t *info)
{
    lcs_status st;
    if ((st = check_mesh(mesh)) != LCS_OK) return st;
    if (!info) return lcs::set_error(LCS_E_ARG, "info is NULL");
    memset(info, 0, sizeof(*info));
    info->dim = mesh->dim;
    info->n_nodes = mesh->n_nodes;
    info->n_cells = mesh->n_cells;
    info->n_boundary_faces = mesh->n_boundary;
    for (int a = 0; a < 3; ++a) {
        info->buckets[a] = mesh->nb[a];
        info->lo[a] = mesh->lo[a];
        info->hi[a] = mesh->hi[a];
    }
    info->device_bytes = mesh->bytes;
    return lcs::clear_error();
}

lcs_status lcs_mesh_locate(lcs_mesh_t mesh, const float *x, int64_t n, int64_t *cell, float *lam,
                           void *stream)
{
    lcs_status st;
    if ((st = check_mesh(mesh)) != LCS_OK) return st;
    if (n < 0 || n > INT_MAX) return lcs::set_error(LCS_E_SHAPE, "n must be in [0, 2^31)");
    if (n == 0) return lcs::clear_error();
    if (!x || !cell) return lcs::set_error(LCS_E_ARG, "x and cell must not be NULL");
    hipError_t e = lcs::launch_mesh_locate(mesh->dim, mesh_dev(mesh), x, n,
                                           reinterpret_cast<long long *>(cell), lam,
                                           (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "mesh locate launch");
    return lcs::clear_error();
}

lcs_status lcs_mesh_velocity_at(lcs_mesh_t mesh, const lcs_mesh_frames_t *frames, const float *x,
                                const double *t, int64_t n, float *u, int64_t *cell, void *stream)
{
    lcs_status st;
    if ((st = check_mesh(mesh)) != LCS_OK) return st;
    if ((st = check_frames(mesh, frames)) != LCS_OK) return st;
    if (n < 0 || n > INT_MAX) return lcs::set_error(LCS_E_SHAPE, "n must be in [0, 2^31)");
    if (n == 0) return lcs::clear_error();
    if (!x || !t || !u) return lcs::set_error(LCS_E_ARG, "x, t and u must not be NULL");
    hipError_t e = lcs::launch_mesh_velocity(mesh->dim, mesh_dev(mesh), frames_dev(mesh, frames), x,
                                             t, n, u, reinterpret_cast<long long *>(cell),
                                             (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "mesh velocity launch");
    return lcs::clear_error();
}

lcs_status lcs_mesh_advect(lcs_mesh_t mesh, const lcs_mesh_frames_t *frames,
                           const lcs_seed_grid_t *seeds, double t0, double T, double dt,
                           float *xf, int64_t *cell, uint8_t *flags, void *stream)
{
    lcs_status st;
    if ((st = check_mesh(mesh)) != LCS_OK) return st;
    if ((st = check_frames(mesh, frames)) != LCS_OK) return st;
    if ((st = lcs::validate_seeds(seeds, mesh->dim)) != LCS_OK) return st;
    if (seeds->periodic_mask)
        return lcs::set_error(LCS_E_UNSUPPORTED, "seed grids over a mesh are not periodic");
    if (!xf) return lcs::set_error(LCS_E_ARG, "xf is NULL");
    int nsteps = 0;
    if ((st = lcs::validate_steps(T, dt, &nsteps)) != LCS_OK) return st;
    const lcs::MeshFramesDev f = frames_dev(mesh, frames);
    const double t1 = t0 + T;
    if (!(std::isfinite(t0) && t0 >= f.t_first && t0 <= f.t_last && t1 >= f.t_first && t1 <= f.t_last))
        return lcs::set_error(LCS_E_TIME_RANGE, "[%g, %g] leaves the frame span [%g, %g]", t0, t1,
                              f.t_first, f.t_last);
    lcs::MeshAdvectArgs A;
    memset(&A, 0, sizeof(A));
    A.m = mesh_dev(mesh);
    A.f = f;
    A.g = lcs::seed_tiling(seeds);
    A.t0 = t0;
    A.dt = dt;
    A.nsteps = nsteps;
    A.ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    A.xf = xf;
    A.cell = reinterpret_cast<long long *>(cell);
    A.flags = flags;
    hipError_t e = lcs::launch_mesh_advect(mesh->dim, A, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "mesh advect launch");
    return lcs::clear_error();
}

lcs_status lcs_mesh_advect_points(lcs_mesh_t mesh, const lcs_mesh_frames_t *frames,
                                  const float *x0, const double *t0, int64_t n, double T,
                                  double dt, float *xf, int64_t *cell, uint8_t *flags,
                                  void *stream)
{
    lcs_status st;
    if ((st = check_mesh(mesh)) != LCS_OK) return st;
    if ((st = check_frames(mesh, frames)) != LCS_OK) return st;
    if (n < 0 || n > INT_MAX) return lcs::set_error(LCS_E_SHAPE, "n must be in [0, 2^31)");
    int nsteps = 0;
    if ((st = lcs::validate_steps(T, dt, &nsteps)) != LCS_OK) return st;
    if (n == 0) return lcs::clear_error();
    if (!x0 || !t0 || !xf) return lcs::set_error(LCS_E_ARG, "x0, t0 and xf must not be NULL");
    lcs::MeshAdvectArgs A;
    memset(&A, 0, sizeof(A));
    A.m = mesh_dev(mesh);
    A.f = frames_dev(mesh, frames);
    A.dt = dt;
    A.nsteps = nsteps;
    A.ns = n;
    A.xf = xf;
    A.cell = reinterpret_cast<long long *>(cell);
    A.flags = flags;
    A.x0 = x0;
    A.t0v = t0;
    A.T = T;
    hipError_t e = lcs::launch_mesh_advect_points(mesh->dim, A, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "mesh advect_points launch");
    return lcs::clear_error();
}

}  // extern "C"
