// api.hip -- the C ABI declared in include/lcs.h: host-side validation,
// work decomposition and launches.  Every argument is checked before anything
// is enqueued.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lcs_internal.h"

namespace {
thread_local char g_err[512] = "";
}

namespace lcs {

lcs_status set_error(lcs_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

lcs_status clear_error()
{
    g_err[0] = '\0';
    return LCS_OK;
}

lcs_status hip_error(hipError_t e, const char *where)
{
    return set_error(LCS_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

}  // namespace lcs

namespace {


bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

constexpr long long kMaxNodes = (1LL << 31) - 1;
constexpr long long kMaxSeeds = (1LL << 31) - 1;

lcs_status check_velocity(const lcs_velocity_t *v)
{
    if (!v) return lcs::set_error(LCS_E_ARG, "velocity descriptor is NULL");
    if (v->dim != 2 && v->dim != 3) return lcs::set_error(LCS_E_ARG, "velocity dim must be 2 or 3 (got %d)", v->dim);
    if (v->layout > LCS_LAYOUT_TPAIR || (v->layout == LCS_LAYOUT_XYZW && v->dim != 3))
        return lcs::set_error(LCS_E_ARG, "velocity layout %u is not valid for %dD", v->layout, v->dim);
    if (v->layout != LCS_LAYOUT_SOA) {
        const uintptr_t align = (v->layout == LCS_LAYOUT_XYZW || v->layout == LCS_LAYOUT_TPAIR)
                                    ? 16u : (v->dim == 2 ? 8u : 4u);
        if (!v->u[0]) return lcs::set_error(LCS_E_ARG, "interleaved frames pointer u[0] is NULL");
        if (reinterpret_cast<uintptr_t>(v->u[0]) % align)
            return lcs::set_error(LCS_E_ARG, "interleaved frames must be %d-byte aligned", (int)align);
    }
    if (v->n_frames < 2) return lcs::set_error(LCS_E_SHAPE, "need at least 2 frames (got %d)", v->n_frames);
    if (!finite_pos(v->dt_frame) || !isfinite(v->t_first))
        return lcs::set_error(LCS_E_ARG, "t_first must be finite and dt_frame > 0");
    if (v->periodic_mask >> v->dim) return lcs::set_error(LCS_E_ARG, "periodic_mask has bits beyond dim");
    long long nodes = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < v->dim) {
            if (v->n[a] < 2) return lcs::set_error(LCS_E_SHAPE, "velocity axis %d needs >= 2 nodes", a);
            if (!finite_pos(v->spacing[a]) || !isfinite(v->origin[a]))
                return lcs::set_error(LCS_E_ARG, "velocity axis %d: bad origin/spacing", a);
            if (v->layout == LCS_LAYOUT_SOA && !v->u[a])
                return lcs::set_error(LCS_E_ARG, "velocity component %d pointer is NULL", a);
        } else if (v->n[a] != 1) {
            return lcs::set_error(LCS_E_SHAPE, "velocity n[%d] must be 1 in %dD", a, v->dim);
        }
        nodes *= v->n[a];
        if (nodes > kMaxNodes) return lcs::set_error(LCS_E_SHAPE, "velocity frame exceeds 2^31-1 nodes");
    }
    // kernels address a frame array (a frame-pair block for TPAIR) with 32-bit
    // byte offsets
    const long long rec = (v->layout == LCS_LAYOUT_SOA) ? 4 :
                          (v->layout == LCS_LAYOUT_XYZW) ? 16 :
                          (v->layout == LCS_LAYOUT_TPAIR) ? 8LL * v->dim : 4LL * v->dim;
    const long long recs = (v->layout == LCS_LAYOUT_TPAIR) ? nodes / v->n[0] * (v->n[0] + 1) : nodes;
    if (recs * rec > (1LL << 32))
        return lcs::set_error(LCS_E_SHAPE, "a velocity frame array exceeds 4 GiB (%lld records x %lld B)",
                              recs, rec);
    return LCS_OK;
}

lcs_status check_seeds(const lcs_seed_grid_t *g, int dim)
{
    if (!g) return lcs::set_error(LCS_E_ARG, "seed grid descriptor is NULL");
    if (g->dim != dim) return lcs::set_error(LCS_E_ARG, "seed grid dim %d != %d", g->dim, dim);
    if (g->periodic_mask >> g->dim) return lcs::set_error(LCS_E_ARG, "seed periodic_mask has bits beyond dim");
    long long ns = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < g->dim) {
            if (g->n[a] < 2) return lcs::set_error(LCS_E_SHAPE, "seed axis %d needs >= 2 seeds", a);
            if (!finite_pos(g->spacing[a]) || !isfinite(g->origin[a]))
                return lcs::set_error(LCS_E_ARG, "seed axis %d: bad origin/spacing", a);
        } else if (g->n[a] != 1) {
            return lcs::set_error(LCS_E_SHAPE, "seed n[%d] must be 1 in %dD", a, g->dim);
        }
        ns *= g->n[a];
        if (ns > kMaxSeeds) return lcs::set_error(LCS_E_SHAPE, "seed grid exceeds 2^31-1 seeds");
    }
    return LCS_OK;
}

// N = T/dt must be a positive integer (to 1e-9 relative), with sign(dt) == sign(T).
lcs_status check_steps(double T, double dt, int *nsteps)
{
    if (!isfinite(T) || !isfinite(dt) || T == 0.0 || dt == 0.0)
        return lcs::set_error(LCS_E_STEP, "T and dt must be finite and non-zero");
    if ((T > 0.0) != (dt > 0.0)) return lcs::set_error(LCS_E_STEP, "sign(dt) must equal sign(T)");
    const double r = T / dt;
    const double N = nearbyint(r);
    if (fabs(r - N) > 1e-9 * fabs(r)) return lcs::set_error(LCS_E_STEP, "T/dt = %.17g is not an integer", r);
    if (N < 1.0 || N > 2147483647.0) return lcs::set_error(LCS_E_STEP, "step count out of range");
    *nsteps = (int)N;
    return LCS_OK;
}

// Seeds must lie inside the closed domain on every non-periodic velocity axis
// (to 1e-9 of the extent); a periodic seed axis needs a periodic velocity axis.
lcs_status check_seed_domain(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds)
{
    for (int a = 0; a < vel->dim; ++a) {
        const bool vper = (vel->periodic_mask >> a) & 1u;
        const bool sper = (seeds->periodic_mask >> a) & 1u;
        if (sper && !vper) return lcs::set_error(LCS_E_ARG, "seed axis %d periodic but velocity axis is not", a);
        if (sper) {
            // the gradient shifts a seam neighbour by the seed period, which is
            // right only when it is the velocity period
            const double Lv = (double)vel->n[a] * vel->spacing[a];
            const double Ls = (double)seeds->n[a] * seeds->spacing[a];
            if (!(fabs(Ls - Lv) <= 1e-9 * Lv))
                return lcs::set_error(LCS_E_ARG, "periodic seed axis %d has period %g, the velocity "
                                      "period is %g", a, Ls, Lv);
        }
        if (vper) continue;
        const double lo = vel->origin[a];
        const double hi = vel->origin[a] + (double)(vel->n[a] - 1) * vel->spacing[a];
        const double s0 = seeds->origin[a];
        const double s1 = seeds->origin[a] + (double)(seeds->n[a] - 1) * seeds->spacing[a];
        const double tol = 1e-9 * (hi - lo);
        if (s0 < lo - tol || s1 > hi + tol)
            return lcs::set_error(LCS_E_SEED_DOMAIN, "seeds on axis %d span [%g, %g] outside [%g, %g]", a,
                        s0, s1, lo, hi);
    }
    return LCS_OK;
}

lcs::VelDev make_vel(const lcs_velocity_t *v)
{
    lcs::VelDev d;
    memset(&d, 0, sizeof(d));
    // TPAIR: a "frame" is a frame-pair block of (n0+1)*n1*n2 records of 2*dim floats
    const bool tpair = (v->layout == LCS_LAYOUT_TPAIR);
    const long long n0r = tpair ? v->n[0] + 1 : v->n[0];
    d.frame_stride = n0r * v->n[1] * v->n[2];
    if (v->layout != LCS_LAYOUT_SOA) {
        d.ilv = tpair ? 2 * v->dim : (v->layout == LCS_LAYOUT_XYZW) ? 4 : v->dim;
        d.ilv_u = v->u[0];
    }
    const uint32_t rec = (v->layout == LCS_LAYOUT_SOA) ? 4u : 4u * (uint32_t)(d.ilv);
    d.sb[0] = rec;
    d.sb[1] = rec * (uint32_t)n0r;
    d.sb[2] = rec * (uint32_t)(n0r * v->n[1]);
    for (int a = 0; a < 3; ++a) {
        d.u[a] = (a < v->dim && v->layout == LCS_LAYOUT_SOA) ? v->u[a] : nullptr;
        d.n[a] = (int)v->n[a];
        d.nf[a] = (float)v->n[a];
        const double inv = 1.0 / v->spacing[a];
        d.oh[a] = (float)v->origin[a];
        d.ol[a] = (float)(v->origin[a] - (double)d.oh[a]);
        d.ih[a] = (float)inv;
        d.il[a] = (float)(inv - (double)d.ih[a]);
        d.lo[a] = (float)v->origin[a];
        d.hi[a] = (float)(v->origin[a] + (double)(v->n[a] - 1) * v->spacing[a]);
        d.origin_d[a] = v->origin[a];
        d.spacing_d[a] = v->spacing[a];
    }
    d.periodic_mask = v->periodic_mask;
    d.n_frames = v->n_frames;
    d.t_first = v->t_first;
    d.dt_frame = v->dt_frame;
    d.inv_dt_frame = 1.0 / v->dt_frame;
    d.t_last = v->t_first + (double)(v->n_frames - 1) * v->dt_frame;
    return d;
}

int ceil_log2(int x)
{
    int b = 0;
    while ((1 << b) < x) ++b;
    return b;
}

lcs::SeedTiling make_tiling(const lcs_seed_grid_t *g)
{
    lcs::SeedTiling t;
    memset(&t, 0, sizeof(t));
    // wave sub-tile: 8x8 in 2D, 4x4x4 in 3D; 4 waves per workgroup as 2x2(x1)
    const int wt2[3] = {8, 8, 1}, wt3[3] = {4, 4, 4};
    const int wg[3] = {2, 2, 1};
    int nb = 1;
    for (int a = 0; a < 3; ++a) {
        t.sn[a] = (int)g->n[a];
        t.s_origin[a] = g->origin[a];
        t.s_spacing[a] = g->spacing[a];
        t.wt[a] = (g->dim == 2) ? wt2[a] : wt3[a];
        t.wg[a] = (a < g->dim) ? wg[a] : 1;
        const int tile = t.wt[a] * t.wg[a];
        t.ntiles[a] = (a < g->dim) ? (int)((g->n[a] + tile - 1) / tile) : 1;
        t.bits[a] = (a < g->dim) ? ceil_log2(t.ntiles[a]) : 0;
        if (t.bits[a] > t.max_bits) t.max_bits = t.bits[a];
        nb *= (1 << t.bits[a]);
    }
    t.n_blocks = nb;
    return t;
}

}  // namespace

namespace lcs {
lcs_status validate_velocity(const lcs_velocity_t *v) { return check_velocity(v); }
lcs_status validate_seeds(const lcs_seed_grid_t *g, int dim) { return check_seeds(g, dim); }
lcs_status validate_steps(double T, double dt, int *nsteps) { return check_steps(T, dt, nsteps); }
lcs_status validate_seed_domain(const lcs_velocity_t *v, const lcs_seed_grid_t *g)
{
    return check_seed_domain(v, g);
}
VelDev velocity_dev(const lcs_velocity_t *v) { return make_vel(v); }
SeedTiling seed_tiling(const lcs_seed_grid_t *g) { return make_tiling(g); }
}  // namespace lcs

// Plan: device state owned by the library for batched launches -- the work
// counter, a capture stream (default priority) and the instantiated graph of
// (counter reset + persistent kernel) together with the key it was captured
// for.  Created by lcs_plan_create, freed by lcs_plan_destroy.
struct lcs_plan {
    int device = -1;
    int *d_counter = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool have_graph = false;
    lcs::BatchArgs key;       // arguments the graph was captured with
    int key_dim = 0;
    int key_grid = 0;
    long long launches = 0;
    long long captures = 0;
    // autotuner: chosen segment length (0 = single launch) per workload key,
    // and the file the choices are read from / appended to (may be empty)
    std::string cache_path;
    std::vector<std::pair<std::string, int>> tuned;
};

namespace {

void drop_graph(lcs_plan *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->have_graph = false;
}

// Autotuner cache: one JSON object per line,
//   {"key": "<workload key>", "segment_steps": S, "ms": [...]}
// later lines for the same key override earlier ones.
void read_tune_cache(lcs_plan *p)
{
    FILE *f = fopen(p->cache_path.c_str(), "r");
    if (!f) return;
    char line[1024], key[512];
    int seg = 0;
    while (fgets(line, sizeof(line), f)) {
        if (sscanf(line, " {\"key\": \"%511[^\"]\", \"segment_steps\": %d", key, &seg) != 2) continue;
        bool found = false;
        for (auto &kv : p->tuned)
            if (kv.first == key) { kv.second = seg; found = true; }
        if (!found) p->tuned.emplace_back(key, seg);
    }
    fclose(f);
}

// Workload key: device architecture, velocity grid and layout, frame count,
// periodicity, seed grid, step count and direction.
std::string tune_key(const lcs_velocity_t *v, const lcs_seed_grid_t *g, int nsteps, double dt,
                     int device)
{
    hipDeviceProp_t prop;
    char arch[64] = "unknown";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
        char *colon = strchr(arch, ':');
        if (colon) *colon = '\0';
    }
    char buf[512];
    snprintf(buf, sizeof(buf), "%s:%dd:grid%lldx%lldx%lld:layout%u:per%u:frames%d:seeds%lldx%lldx%lld:"
             "steps%d%s", arch, v->dim, (long long)v->n[0], (long long)v->n[1], (long long)v->n[2],
             v->layout, v->periodic_mask, v->n_frames, (long long)g->n[0], (long long)g->n[1],
             (long long)g->n[2], nsteps, dt < 0 ? "b" : "f");
    return buf;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch timing: event pairs per kernel launch, kept until queried or cleared.
// ---------------------------------------------------------------------------
namespace {
struct TimedLaunch {
    std::string name;
    hipEvent_t ev[2];
};
std::mutex g_timing_mu;
bool g_timing_on = false;
std::vector<TimedLaunch> g_timing;

void timing_clear_locked()
{
    for (auto &t : g_timing) {
        if (t.ev[0]) (void)hipEventDestroy(t.ev[0]);
        if (t.ev[1]) (void)hipEventDestroy(t.ev[1]);
    }
    g_timing.clear();
}
}  // namespace

namespace lcs {
LaunchTimer::LaunchTimer(const char *name, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_timing_mu);
    if (!g_timing_on) return;
    TimedLaunch t;
    t.name = name;
    t.ev[0] = t.ev[1] = nullptr;
    if (hipEventCreate(&t.ev[0]) != hipSuccess || hipEventCreate(&t.ev[1]) != hipSuccess ||
        hipEventRecord(t.ev[0], s) != hipSuccess) {
        if (t.ev[0]) (void)hipEventDestroy(t.ev[0]);
        if (t.ev[1]) (void)hipEventDestroy(t.ev[1]);
        return;
    }
    slot = (int)g_timing.size();
    g_timing.push_back(t);
}

void LaunchTimer::stop(hipStream_t s)
{
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_timing_mu);
    if (slot < (int)g_timing.size()) (void)hipEventRecord(g_timing[slot].ev[1], s);
    slot = -1;
}
}  // namespace lcs

extern "C" {

lcs_status lcs_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_timing_mu);
    timing_clear_locked();
    g_timing_on = (on != 0);
    return lcs::clear_error();
}

lcs_status lcs_timing_query(const char *kernel, int64_t *launches, double *total_ms)
{
    if (!kernel || !launches || !total_ms)
        return lcs::set_error(LCS_E_ARG, "kernel, launches and total_ms must not be NULL");
    std::lock_guard<std::mutex> lk(g_timing_mu);
    long long n = 0;
    double ms = 0.0;
    for (auto &t : g_timing) {
        if (t.name != kernel) continue;
        float e = 0.0f;
        const hipError_t r = hipEventElapsedTime(&e, t.ev[0], t.ev[1]);
        if (r != hipSuccess) return lcs::hip_error(r, "timing query (synchronize first)");
        ++n;
        ms += e;
    }
    *launches = n;
    *total_ms = ms;
    return lcs::clear_error();
}

}  // extern "C"

extern "C" {

lcs_status lcs_plan_create(lcs_plan_t *plan, const char *autotune_cache_path)
{
    if (!plan) return lcs::set_error(LCS_E_ARG, "plan pointer is NULL");
    *plan = nullptr;
    lcs_plan *p = new (std::nothrow) lcs_plan();
    if (!p) return lcs::set_error(LCS_E_ARG, "out of host memory");
    if (autotune_cache_path && autotune_cache_path[0]) {
        p->cache_path = autotune_cache_path;
        read_tune_cache(p);
    }
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipMalloc((void **)&p->d_counter, lcs::kBatchCounters * sizeof(int));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (p->d_counter) (void)hipFree(p->d_counter);
        delete p;
        return lcs::hip_error(e, "lcs_plan_create");
    }
    *plan = p;
    return lcs::clear_error();
}

lcs_status lcs_plan_destroy(lcs_plan_t plan)
{
    if (!plan) return lcs::clear_error();
    (void)hipStreamSynchronize(plan->cap_stream);
    drop_graph(plan);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    if (plan->d_counter) (void)hipFree(plan->d_counter);
    delete plan;
    return lcs::clear_error();
}

lcs_status lcs_plan_stats(lcs_plan_t plan, int64_t *graph_launches, int64_t *graph_captures)
{
    if (!plan) return lcs::set_error(LCS_E_ARG, "plan is NULL");
    if (graph_launches) *graph_launches = plan->launches;
    if (graph_captures) *graph_captures = plan->captures;
    return lcs::clear_error();
}

const char *lcs_last_error(void) { return g_err; }

int32_t lcs_version(void) { return 100; }

lcs_status lcs_sync_status(void *stream)
{
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "hipStreamSynchronize");
    e = hipGetLastError();
    if (e != hipSuccess) return lcs::hip_error(e, "pending error");
    return lcs::clear_error();
}

lcs_status lcs_frames_interleave(const lcs_velocity_t *soa, uint32_t layout, int32_t f_first,
                                 int32_t f_count, float *out, lcs_velocity_t *out_desc,
                                 void *stream)
{
    lcs_status st;
    if ((st = check_velocity(soa)) != LCS_OK) return st;
    if (soa->layout != LCS_LAYOUT_SOA) return lcs::set_error(LCS_E_ARG, "source frames must be LCS_LAYOUT_SOA");
    if (layout != LCS_LAYOUT_XYZ && layout != LCS_LAYOUT_TPAIR &&
        !(layout == LCS_LAYOUT_XYZW && soa->dim == 3))
        return lcs::set_error(LCS_E_ARG, "target layout must be LCS_LAYOUT_XYZ, TPAIR (or XYZW in 3D)");
    if (!out || !out_desc) return lcs::set_error(LCS_E_ARG, "out and out_desc must not be NULL");
    if (f_first < 0 || f_count < 2 || (long long)f_first + f_count > soa->n_frames)
        return lcs::set_error(LCS_E_SHAPE, "frame span [%d, %d) outside [0, %d) or shorter than 2",
                              f_first, f_first + f_count, soa->n_frames);
    const int S = (layout == LCS_LAYOUT_XYZW) ? 4 : soa->dim;
    const uintptr_t align = (layout == LCS_LAYOUT_XYZ) ? (soa->dim == 2 ? 8u : 4u) : 16u;
    if (reinterpret_cast<uintptr_t>(out) % align)
        return lcs::set_error(LCS_E_ARG, "out must be %d-byte aligned", (int)align);
    lcs_velocity_t desc = *soa;
    desc.layout = layout;
    desc.n_frames = f_count;
    desc.u[0] = out;
    desc.u[1] = desc.u[2] = nullptr;
    if ((st = check_velocity(&desc)) != LCS_OK) return st;   // size limits of the target layout
    const long long nodes = soa->n[0] * soa->n[1] * soa->n[2];
    hipError_t e;
    if (layout == LCS_LAYOUT_TPAIR) {
        const int n[3] = {(int)soa->n[0], (int)soa->n[1], (int)soa->n[2]};
        e = lcs::launch_interleave_tpair(soa->dim, soa->u, n, f_count, f_first, out,
                                         (hipStream_t)stream);
    } else {
        e = lcs::launch_interleave(soa->dim, S, soa->u, nodes, f_count, f_first, out,
                                   (hipStream_t)stream);
    }
    if (e != hipSuccess) return lcs::hip_error(e, "interleave launch");
    *out_desc = *soa;
    out_desc->layout = layout;
    out_desc->n_frames = f_count;
    out_desc->t_first = soa->t_first + (double)f_first * soa->dt_frame;
    out_desc->u[0] = out;
    out_desc->u[1] = nullptr;
    out_desc->u[2] = nullptr;
    return lcs::clear_error();
}

int64_t lcs_frames_interleave_floats(const lcs_velocity_t *soa, uint32_t layout, int32_t f_count)
{
    if (!soa || (soa->dim != 2 && soa->dim != 3) || f_count < 2) return -1;
    const long long nodes = soa->n[0] * soa->n[1] * soa->n[2];
    switch (layout) {
    case LCS_LAYOUT_XYZ: return (int64_t)f_count * nodes * soa->dim;
    case LCS_LAYOUT_XYZW: return soa->dim == 3 ? (int64_t)f_count * nodes * 4 : -1;
    case LCS_LAYOUT_TPAIR:
        return (int64_t)(f_count - 1) * (soa->n[0] + 1) * soa->n[1] * soa->n[2] * 2 * soa->dim;
    default: return -1;
    }
}

lcs_status lcs_advect(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, double t0,
                      double T, double dt, float *xf, int64_t *cell, uint8_t *flags, void *stream)
{
    lcs_status st;
    if ((st = check_velocity(vel)) != LCS_OK) return st;
    if ((st = check_seeds(seeds, vel->dim)) != LCS_OK) return st;
    if (!xf) return lcs::set_error(LCS_E_ARG, "xf is NULL");
    int nsteps = 0;
    if ((st = check_steps(T, dt, &nsteps)) != LCS_OK) return st;
    const double t_last = vel->t_first + (double)(vel->n_frames - 1) * vel->dt_frame;
    const double t1 = t0 + T;
    if (!(isfinite(t0) && t0 >= vel->t_first && t0 <= t_last && t1 >= vel->t_first && t1 <= t_last))
        return lcs::set_error(LCS_E_TIME_RANGE, "[%g, %g] leaves the frame span [%g, %g]", t0, t1,
                    vel->t_first, t_last);
    if ((st = check_seed_domain(vel, seeds)) != LCS_OK) return st;
    lcs::AdvectArgs A;
    memset(&A, 0, sizeof(A));
    A.v = make_vel(vel);
    A.g = make_tiling(seeds);
    A.t0 = t0;
    A.dt = dt;
    A.nsteps = nsteps;
    A.ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    A.xf = xf;
    A.cell = reinterpret_cast<long long *>(cell);
    A.flags = flags;
    hipError_t e = lcs::launch_advect_grid(vel->dim, A, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "advect launch");
    return lcs::clear_error();
}

lcs_status lcs_advect_ab(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, int32_t order,
                         double t0, double T, double dt, float *xf, int64_t *cell, uint8_t *flags,
                         void *stream)
{
    lcs_status st;
    if (order < 2 || order > 4) return lcs::set_error(LCS_E_ARG, "order must be 2, 3 or 4");
    if ((st = check_velocity(vel)) != LCS_OK) return st;
    if ((st = check_seeds(seeds, vel->dim)) != LCS_OK) return st;
    if (!xf) return lcs::set_error(LCS_E_ARG, "xf is NULL");
    int nsteps = 0;
    if ((st = check_steps(T, dt, &nsteps)) != LCS_OK) return st;
    const double t_last = vel->t_first + (double)(vel->n_frames - 1) * vel->dt_frame;
    const double t1 = t0 + T;
    if (!(isfinite(t0) && t0 >= vel->t_first && t0 <= t_last && t1 >= vel->t_first && t1 <= t_last))
        return lcs::set_error(LCS_E_TIME_RANGE, "[%g, %g] leaves the frame span [%g, %g]", t0, t1,
                    vel->t_first, t_last);
    if ((st = check_seed_domain(vel, seeds)) != LCS_OK) return st;
    lcs::AdvectArgs A;
    memset(&A, 0, sizeof(A));
    A.v = make_vel(vel);
    A.g = make_tiling(seeds);
    A.t0 = t0;
    A.dt = dt;
    A.nsteps = nsteps;
    A.ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    A.xf = xf;
    A.cell = reinterpret_cast<long long *>(cell);
    A.flags = flags;
    hipError_t e = lcs::launch_advect_ab(vel->dim, order, A, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "advect_ab launch");
    return lcs::clear_error();
}

lcs_status lcs_advect_aux(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds,
                          const double *delta, double t0, double T, double dt, float *xa_hi,
                          float *xa_lo, uint8_t *flags, void *stream)
{
    lcs_status st;
    if ((st = check_velocity(vel)) != LCS_OK) return st;
    if ((st = check_seeds(seeds, vel->dim)) != LCS_OK) return st;
    if (!delta) return lcs::set_error(LCS_E_ARG, "delta is NULL");
    for (int a = 0; a < vel->dim; ++a)
        if (!finite_pos(delta[a])) return lcs::set_error(LCS_E_ARG, "delta[%d] must be > 0", a);
    if (!xa_hi || !xa_lo) return lcs::set_error(LCS_E_ARG, "xa_hi and xa_lo must not be NULL");
    int nsteps = 0;
    if ((st = check_steps(T, dt, &nsteps)) != LCS_OK) return st;
    const double t_last = vel->t_first + (double)(vel->n_frames - 1) * vel->dt_frame;
    const double t1 = t0 + T;
    if (!(isfinite(t0) && t0 >= vel->t_first && t0 <= t_last && t1 >= vel->t_first && t1 <= t_last))
        return lcs::set_error(LCS_E_TIME_RANGE, "[%g, %g] leaves the frame span [%g, %g]", t0, t1,
                    vel->t_first, t_last);
    if ((st = check_seed_domain(vel, seeds)) != LCS_OK) return st;
    lcs::AuxArgs A;
    memset(&A, 0, sizeof(A));
    A.a.v = make_vel(vel);
    A.a.g = make_tiling(seeds);
    A.a.t0 = t0;
    A.a.dt = dt;
    A.a.nsteps = nsteps;
    A.a.ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    A.a.flags = flags;
    for (int a = 0; a < vel->dim; ++a) A.delta[a] = delta[a];
    A.xa_hi = xa_hi;
    A.xa_lo = xa_lo;
    hipError_t e = lcs::launch_advect_aux(vel->dim, A, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "advect_aux launch");
    return lcs::clear_error();
}

lcs_status lcs_cg_aux(const lcs_seed_grid_t *seeds, const double *delta, const float *xa_hi,
                      const float *xa_lo, const uint8_t *flags, double *C, uint8_t *stencil_flags,
                      void *stream)
{
    if (!seeds) return lcs::set_error(LCS_E_ARG, "seed grid descriptor is NULL");
    lcs_status st;
    if ((st = check_seeds(seeds, seeds->dim)) != LCS_OK) return st;
    if (seeds->dim != 2 && seeds->dim != 3) return lcs::set_error(LCS_E_ARG, "dim must be 2 or 3");
    if (!delta) return lcs::set_error(LCS_E_ARG, "delta is NULL");
    for (int a = 0; a < seeds->dim; ++a)
        if (!finite_pos(delta[a])) return lcs::set_error(LCS_E_ARG, "delta[%d] must be > 0", a);
    if (!xa_hi || !xa_lo || !C) return lcs::set_error(LCS_E_ARG, "xa_hi, xa_lo and C must not be NULL");
    lcs::CgAuxArgs A;
    memset(&A, 0, sizeof(A));
    A.dim = seeds->dim;
    A.ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    for (int a = 0; a < seeds->dim; ++a) A.delta[a] = delta[a];
    A.xa_hi = xa_hi;
    A.xa_lo = xa_lo;
    A.flags = flags;
    A.C = C;
    A.sflags = stencil_flags;
    hipError_t e = lcs::launch_cg_aux(A, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "cg_aux launch");
    return lcs::clear_error();
}

lcs_status lcs_cg_eig(int32_t dim, int64_t n, const double *C, double *evals, double *evecs,
                      void *stream)
{
    if (dim != 2 && dim != 3) return lcs::set_error(LCS_E_ARG, "dim must be 2 or 3");
    if (n < 0 || n > kMaxSeeds) return lcs::set_error(LCS_E_SHAPE, "n out of range");
    if (!C) return lcs::set_error(LCS_E_ARG, "C is NULL");
    if (!evals && !evecs) return lcs::set_error(LCS_E_ARG, "evals and evecs are both NULL");
    if (n == 0) return lcs::clear_error();
    hipError_t e = lcs::launch_eig(dim, n, C, evals, evecs, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "eig launch");
    return lcs::clear_error();
}

lcs_status lcs_advect_snapshots(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, double t0,
                                double dt, int32_t n_snap, const int32_t *snap_steps, float *xf,
                                uint8_t *flags, int32_t *steps_done, void *stream)
{
    lcs_status st;
    if ((st = check_velocity(vel)) != LCS_OK) return st;
    if ((st = check_seeds(seeds, vel->dim)) != LCS_OK) return st;
    if (!xf || !snap_steps) return lcs::set_error(LCS_E_ARG, "xf and snap_steps must not be NULL");
    if (n_snap < 1 || n_snap > LCS_MAX_SNAPSHOTS)
        return lcs::set_error(LCS_E_SHAPE, "n_snap must be in [1, %d]", LCS_MAX_SNAPSHOTS);
    for (int k = 0; k < n_snap; ++k)
        if (snap_steps[k] < 1 || (k > 0 && snap_steps[k] <= snap_steps[k - 1]))
            return lcs::set_error(LCS_E_ARG, "snap_steps must be >= 1 and strictly increasing");
    if (!isfinite(dt) || dt == 0.0) return lcs::set_error(LCS_E_STEP, "dt must be finite and non-zero");
    const double T = dt * (double)snap_steps[n_snap - 1];
    const double t_last = vel->t_first + (double)(vel->n_frames - 1) * vel->dt_frame;
    const double t1 = t0 + T;
    if (!(isfinite(t0) && t0 >= vel->t_first && t0 <= t_last && t1 >= vel->t_first && t1 <= t_last))
        return lcs::set_error(LCS_E_TIME_RANGE, "[%g, %g] leaves the frame span [%g, %g]", t0, t1,
                    vel->t_first, t_last);
    if ((st = check_seed_domain(vel, seeds)) != LCS_OK) return st;
    lcs::SnapArgs A;
    memset(&A, 0, sizeof(A));
    A.a.v = make_vel(vel);
    A.a.g = make_tiling(seeds);
    A.a.t0 = t0;
    A.a.dt = dt;
    A.a.nsteps = snap_steps[n_snap - 1];
    A.a.ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    A.n_snap = n_snap;
    for (int k = 0; k < n_snap; ++k) A.steps[k] = snap_steps[k];
    A.xf = xf;
    A.flags = flags;
    A.steps_done = steps_done;
    hipError_t e = lcs::launch_advect_snap(vel->dim, A, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "advect_snapshots launch");
    return lcs::clear_error();
}

namespace {
constexpr long long kEarlyHeader = 1024;         // counter (aligned region)
constexpr long long kEarlyEntryBytes = 7 * 3 * 8;

long long early_list_bytes(long long ns) { return ((8 * ns + 255) / 256) * 256; }
}  // namespace

int64_t lcs_ftle_early_workspace_bytes(const lcs_seed_grid_t *seeds)
{
    if (!seeds || check_seeds(seeds, seeds->dim) != LCS_OK) return -1;
    const long long ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    return kEarlyHeader + early_list_bytes(ns) + kEarlyEntryBytes * ns;
}

lcs_status lcs_ftle_early(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, double t0,
                          double dt, int32_t nsteps, const float *xf, const int32_t *steps_done,
                          double *lambda_max, double *ftle, double *t_eff, void *workspace,
                          int64_t workspace_bytes, void *stream)
{
    lcs_status st;
    if ((st = check_velocity(vel)) != LCS_OK) return st;
    if ((st = check_seeds(seeds, vel->dim)) != LCS_OK) return st;
    if (!xf || !steps_done || !ftle || !workspace)
        return lcs::set_error(LCS_E_ARG, "xf, steps_done, ftle and workspace must not be NULL");
    if (nsteps < 1) return lcs::set_error(LCS_E_STEP, "nsteps must be >= 1");
    if (!isfinite(dt) || dt == 0.0) return lcs::set_error(LCS_E_STEP, "dt must be finite and non-zero");
    const double t_last = vel->t_first + (double)(vel->n_frames - 1) * vel->dt_frame;
    const double t1 = t0 + dt * (double)nsteps;
    if (!(isfinite(t0) && t0 >= vel->t_first && t0 <= t_last && t1 >= vel->t_first && t1 <= t_last))
        return lcs::set_error(LCS_E_TIME_RANGE, "[%g, %g] leaves the frame span [%g, %g]", t0, t1,
                    vel->t_first, t_last);
    if ((st = check_seed_domain(vel, seeds)) != LCS_OK) return st;
    const long long ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    const long long fixed = kEarlyHeader + early_list_bytes(ns);
    if (workspace_bytes < fixed + kEarlyEntryBytes)
        return lcs::set_error(LCS_E_ARG, "workspace needs at least %lld bytes",
                              fixed + kEarlyEntryBytes);
    long long chunk = (workspace_bytes - fixed) / kEarlyEntryBytes;
    if (chunk > ns) chunk = ns;
    char *base = static_cast<char *>(workspace);
    lcs::EarlyArgs E;
    memset(&E, 0, sizeof(E));
    E.dim = seeds->dim;
    for (int a = 0; a < 3; ++a) {
        E.n[a] = (int)seeds->n[a];
        E.h[a] = seeds->spacing[a];
    }
    E.periodic_mask = seeds->periodic_mask;
    E.ns = ns;
    E.nsteps = nsteps;
    E.dt = dt;
    E.xf = xf;
    E.steps_done = steps_done;
    E.lam = lambda_max;
    E.ftle = ftle;
    E.t_eff = t_eff;
    E.counter = reinterpret_cast<int *>(base);
    E.list = reinterpret_cast<int *>(base + kEarlyHeader);
    E.pos = reinterpret_cast<double *>(base + fixed);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = lcs::launch_fill_u32(reinterpret_cast<uint32_t *>(E.counter), 1, 0u, s);
    if (e == hipSuccess) e = lcs::launch_early_mark(E, s);
    int count = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&count, E.counter, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return lcs::hip_error(e, "ftle_early mark");
    lcs::EarlyAdvArgs A;
    memset(&A, 0, sizeof(A));
    A.v = make_vel(vel);
    for (int a = 0; a < 3; ++a) {
        A.s_origin[a] = seeds->origin[a];
        A.s_spacing[a] = seeds->spacing[a];
        A.n[a] = (int)seeds->n[a];
    }
    A.periodic_mask = seeds->periodic_mask;
    A.t0 = t0;
    A.dt = dt;
    A.list = E.list;
    A.pos = E.pos;
    for (long long first = 0; first < count; first += chunk) {
        const int c = (int)((count - first < chunk) ? count - first : chunk);
        e = lcs::launch_early_advect(vel->dim, A, (int)first, c, s);
        if (e == hipSuccess) e = lcs::launch_early_cg(E, (int)first, c, s);
        if (e != hipSuccess) return lcs::hip_error(e, "ftle_early pass");
    }
    return lcs::clear_error();
}

lcs_status lcs_advect_batched(lcs_plan_t plan, const lcs_velocity_t *vel,
                              const lcs_seed_grid_t *seeds, const lcs_window_t *windows,
                              int32_t n_windows, double dt, float *xf, int64_t *cell,
                              uint8_t *flags, void *stream)
{
    lcs_status st;
    if (!plan) return lcs::set_error(LCS_E_ARG, "plan is NULL (create one with lcs_plan_create)");
    if ((st = check_velocity(vel)) != LCS_OK) return st;
    if ((st = check_seeds(seeds, vel->dim)) != LCS_OK) return st;
    if (!xf || !windows) return lcs::set_error(LCS_E_ARG, "xf and windows must not be NULL");
    if (n_windows < 1 || n_windows > lcs::kMaxWindows)
        return lcs::set_error(LCS_E_SHAPE, "n_windows must be in [1, %d]", lcs::kMaxWindows);
    if ((st = check_seed_domain(vel, seeds)) != LCS_OK) return st;
    const double t_last = vel->t_first + (double)(vel->n_frames - 1) * vel->dt_frame;
    lcs::BatchArgs A;
    memset(&A, 0, sizeof(A));
    for (int w = 0; w < n_windows; ++w) {
        int nsteps = 0;
        if ((st = check_steps(windows[w].T, dt, &nsteps)) != LCS_OK) return st;
        const double t0 = windows[w].t0, t1 = t0 + windows[w].T;
        if (!(isfinite(t0) && t0 >= vel->t_first && t0 <= t_last && t1 >= vel->t_first &&
              t1 <= t_last))
            return lcs::set_error(LCS_E_TIME_RANGE, "window %d [%g, %g] leaves the frame span [%g, %g]", w,
                        t0, t1, vel->t_first, t_last);
        A.win[w].t0 = t0;
        A.win[w].nsteps = nsteps;
        A.win[w].out_index = w;
    }
    // earliest start first (stable): the blocks working at any moment then
    // hold tiles of one or two windows that started together and advance
    // together, so they read the same few frame pairs, which stay in L2 and
    // the MALL instead of every window's frames streaming from HBM at once
    for (int i = 1; i < n_windows; ++i) {
        lcs::WindowDev x = A.win[i];
        int j = i - 1;
        while (j >= 0 && A.win[j].t0 > x.t0) {
            A.win[j + 1] = A.win[j];
            --j;
        }
        A.win[j + 1] = x;
    }
    A.v = make_vel(vel);
    A.g = make_tiling(seeds);
    A.dt = dt;
    A.ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    A.n_windows = n_windows;
    const long long items = (long long)n_windows * A.g.n_blocks;
    if (items > 2147483647LL) return lcs::set_error(LCS_E_SHAPE, "too many (window, tile) items");
    A.total_items = (int)items;
    A.counter = plan->d_counter;
    A.xf = xf;
    A.cell = reinterpret_cast<long long *>(cell);
    A.flags = flags;

    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return lcs::hip_error(e, "hipGetDevice");
    if (dev != plan->device) return lcs::set_error(LCS_E_ARG, "plan was created on device %d, current is %d",
                                         plan->device, dev);
    int n_cu = 0;
    e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return lcs::hip_error(e, "hipDeviceGetAttribute");
    // a whole number of blocks per XCD (each XCD's blocks drain its own share)
    int grid = n_cu * lcs::batched_blocks_per_cu(vel->dim);
    grid = (grid + lcs::kBatchCounters - 1) / lcs::kBatchCounters * lcs::kBatchCounters;

    const bool same = plan->have_graph && plan->key_dim == vel->dim && plan->key_grid == grid &&
                      memcmp(&plan->key, &A, sizeof(A)) == 0;
    if (!same) {
        drop_graph(plan);
        // capture (counter reset, persistent kernel) on the plan's own stream
        e = hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return lcs::hip_error(e, "hipStreamBeginCapture");
        hipError_t e1 = lcs::launch_reset_counter(plan->d_counter, plan->cap_stream);
        hipError_t e2 = lcs::launch_advect_batched(vel->dim, A, grid, plan->cap_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(plan->cap_stream, &g);
        if (e1 != hipSuccess || e2 != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return lcs::hip_error(e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e), "graph capture");
        }
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return lcs::hip_error(e, "hipGraphInstantiate");
        }
        plan->graph = g;
        plan->exec = x;
        plan->have_graph = true;
        plan->key = A;
        plan->key_dim = vel->dim;
        plan->key_grid = grid;
        plan->captures++;
    }
    e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "hipGraphLaunch");
    plan->launches++;
    return lcs::clear_error();
}

}  // extern "C"

namespace {

struct SortedLayout {
    lcs::SortKeys sk;
    long long bytes;
};

long long align256(long long x) { return (x + 255) / 256 * 256; }

// Bin geometry and workspace size of lcs_advect_sorted; with base != NULL the
// state buffers and sort arrays are carved from it.
SortedLayout sorted_layout(const lcs_velocity_t *vel, long long n, char *base, lcs::TracerState *st,
                           int order = 0)
{
    SortedLayout L;
    memset(&L, 0, sizeof(L));
    // bin edge in cells: the finest whose Morton keys fit in kMaxBinKeyBits bits
    long long bc = 1;
    for (;;) {
        int key_bits = 0;
        for (int a = 0; a < vel->dim; ++a) key_bits += ceil_log2((int)((vel->n[a] + bc - 1) / bc));
        if (key_bits <= lcs::kMaxBinKeyBits || bc >= (1LL << 20)) break;
        bc *= 2;
    }
    long long nk = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < vel->dim) {
            L.sk.nb[a] = (int)((vel->n[a] + bc - 1) / bc);
            L.sk.bits[a] = ceil_log2(L.sk.nb[a]);
            L.sk.inv_bin[a] = (float)(1.0 / ((double)bc * vel->spacing[a]));
            L.sk.origin[a] = (float)vel->origin[a];
        } else {
            L.sk.nb[a] = 1;
        }
        if (L.sk.bits[a] > L.sk.max_bits) L.sk.max_bits = L.sk.bits[a];
        nk <<= L.sk.bits[a];
    }
    L.sk.n_keys = nk;
    long long off = 0;
    auto take = [&](long long bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    for (int b = 0; b < 2; ++b) {
        for (int a = 0; a < 3; ++a) {
            char *ph = (a < vel->dim) ? take(4 * n) : nullptr;
            char *pl = (a < vel->dim) ? take(4 * n) : nullptr;
            if (st) {
                st[b].xh[a] = reinterpret_cast<float *>(ph);
                st[b].xl[a] = reinterpret_cast<float *>(pl);
            }
        }
        char *pi = take(4 * n);
        char *pf = take(n);
        if (st) {
            st[b].idx = reinterpret_cast<int *>(pi);
            st[b].flag = reinterpret_cast<uint8_t *>(pf);
        }
        for (int q = 0; q < 9; ++q) {
            char *ph = (order > 0 && q < 3 * vel->dim) ? take(4 * n) : nullptr;
            if (st) st[b].hist[q] = reinterpret_cast<float *>(ph);
        }
    }
    L.sk.keys = reinterpret_cast<uint32_t *>(take(4 * n));
    L.sk.perm = reinterpret_cast<uint32_t *>(take(4 * n));
    L.sk.rank = reinterpret_cast<uint32_t *>(take(4 * n));
    L.sk.counts = reinterpret_cast<uint32_t *>(take(4 * nk));
    L.sk.block_sums = reinterpret_cast<uint32_t *>(take(4 * ((nk + 1023) / 1024 + 1)));
    L.bytes = off;
    return L;
}

}  // namespace

extern "C" {

int64_t lcs_advect_sorted_workspace_bytes(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds)
{
    if (check_velocity(vel) != LCS_OK || check_seeds(seeds, vel->dim) != LCS_OK) return 0;
    const long long n = seeds->n[0] * seeds->n[1] * seeds->n[2];
    return sorted_layout(vel, n, nullptr, nullptr).bytes;
}

int64_t lcs_advect_ab_sorted_workspace_bytes(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds)
{
    if (check_velocity(vel) != LCS_OK || check_seeds(seeds, vel->dim) != LCS_OK) return 0;
    const long long n = seeds->n[0] * seeds->n[1] * seeds->n[2];
    return sorted_layout(vel, n, nullptr, nullptr, 4).bytes;
}

}  // extern "C"

namespace {

// Re-bundled advection with RK4 (order 0) or Adams-Bashforth (order 2..4), of
// the seeds or (delta != NULL) of the 2*dim auxiliary points of every seed,
// whose outputs are two-floats (xf high, xf_lo low parts).
lcs_status advect_sorted_impl(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, int order,
                              double t0, double T, double dt, int32_t segment_steps, float *xf,
                              int64_t *cell, uint8_t *flags, void *workspace,
                              int64_t workspace_bytes, void *stream, const double *delta = nullptr,
                              float *xf_lo = nullptr)
{
    lcs_status st;
    if ((st = check_velocity(vel)) != LCS_OK) return st;
    if ((st = check_seeds(seeds, vel->dim)) != LCS_OK) return st;
    if (!xf || !workspace) return lcs::set_error(LCS_E_ARG, "xf and workspace must not be NULL");
    if (delta) {
        for (int a = 0; a < vel->dim; ++a)
            if (!finite_pos(delta[a])) return lcs::set_error(LCS_E_ARG, "delta[%d] must be > 0", a);
        if (!xf_lo) return lcs::set_error(LCS_E_ARG, "xa_hi and xa_lo must not be NULL");
    }
    if (segment_steps < 0) return lcs::set_error(LCS_E_ARG, "segment_steps must be >= 0");
    int nsteps = 0;
    if ((st = check_steps(T, dt, &nsteps)) != LCS_OK) return st;
    const double t_last = vel->t_first + (double)(vel->n_frames - 1) * vel->dt_frame;
    const double t1 = t0 + T;
    if (!(isfinite(t0) && t0 >= vel->t_first && t0 <= t_last && t1 >= vel->t_first && t1 <= t_last))
        return lcs::set_error(LCS_E_TIME_RANGE, "[%g, %g] leaves the frame span [%g, %g]", t0, t1,
                              vel->t_first, t_last);
    if ((st = check_seed_domain(vel, seeds)) != LCS_OK) return st;
    const long long ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    const long long n = delta ? 2LL * vel->dim * ns : ns;
    if (n > kMaxSeeds) return lcs::set_error(LCS_E_SHAPE, "more than 2^31-1 tracers");
    lcs::TracerState bufs[2];
    memset(bufs, 0, sizeof(bufs));
    const SortedLayout need = sorted_layout(vel, n, nullptr, nullptr, order);
    if (workspace_bytes < need.bytes)
        return lcs::set_error(LCS_E_SHAPE, "workspace of %lld bytes is smaller than the %lld needed",
                              (long long)workspace_bytes, need.bytes);
    if (need.sk.n_keys > (1LL << 30)) return lcs::set_error(LCS_E_SHAPE, "velocity grid too large to bin");
    const SortedLayout L = sorted_layout(vel, n, static_cast<char *>(workspace), bufs, order);
    const int seg = segment_steps > 0 ? segment_steps : 50;
    hipStream_t s = (hipStream_t)stream;

    lcs::SegmentArgs A;
    memset(&A, 0, sizeof(A));
    A.v = make_vel(vel);
    A.g = make_tiling(seeds);
    A.t0 = t0;
    A.dt = dt;
    A.n = n;
    A.sk = L.sk;
    A.xf = xf;
    A.xf_lo = xf_lo;
    A.cell = reinterpret_cast<long long *>(cell);
    A.flags = flags;
    A.order = order;
    A.st = bufs[0];
    if (delta) {
        A.aux = 1;
        A.ns_seeds = ns;
        for (int a = 0; a < vel->dim; ++a) A.delta[a] = delta[a];
    }
    // the state lives in bufs[cur] in the order of the last histogram; a sort
    // builds the permutation, and the next segment reads bufs[cur] through it
    // and writes bufs[1 - cur] in sorted order
    hipError_t e = lcs::launch_fill_u32(L.sk.counts, L.sk.n_keys, 0u, s);
    if (e == hipSuccess) e = lcs::launch_rebundle_init(vel->dim, A, s);
    if (e == hipSuccess) e = lcs::launch_rebundle_sort(A, s);
    int cur = 0;
    for (int n0 = 0; n0 < nsteps && e == hipSuccess; n0 += seg) {
        A.st = bufs[cur];
        A.out = bufs[1 - cur];
        A.n_begin = n0;
        A.n_end = (nsteps - n0 < seg) ? nsteps : n0 + seg;
        A.last = (A.n_end == nsteps) ? 1 : 0;
        e = lcs::launch_rebundle_segment(vel->dim, A, s);
        if (!A.last && e == hipSuccess) {
            e = lcs::launch_rebundle_sort(A, s);
            cur = 1 - cur;
        }
    }
    if (e != hipSuccess) return lcs::hip_error(e, "advect_sorted launch");
    return lcs::clear_error();
}

}  // namespace

extern "C" {

lcs_status lcs_advect_sorted(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, double t0,
                             double T, double dt, int32_t segment_steps, float *xf, int64_t *cell,
                             uint8_t *flags, void *workspace, int64_t workspace_bytes, void *stream)
{
    return advect_sorted_impl(vel, seeds, 0, t0, T, dt, segment_steps, xf, cell, flags, workspace,
                              workspace_bytes, stream);
}

lcs_status lcs_advect_ab_sorted(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds,
                                int32_t order, double t0, double T, double dt,
                                int32_t segment_steps, float *xf, int64_t *cell, uint8_t *flags,
                                void *workspace, int64_t workspace_bytes, void *stream)
{
    if (order < 2 || order > 4) return lcs::set_error(LCS_E_ARG, "order must be 2, 3 or 4");
    return advect_sorted_impl(vel, seeds, order, t0, T, dt, segment_steps, xf, cell, flags,
                              workspace, workspace_bytes, stream);
}

int64_t lcs_advect_aux_sorted_workspace_bytes(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds)
{
    if (check_velocity(vel) != LCS_OK || check_seeds(seeds, vel->dim) != LCS_OK) return 0;
    const long long n = 2LL * vel->dim * seeds->n[0] * seeds->n[1] * seeds->n[2];
    return sorted_layout(vel, n, nullptr, nullptr).bytes;
}

lcs_status lcs_advect_aux_sorted(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds,
                                 const double *delta, double t0, double T, double dt,
                                 int32_t segment_steps, float *xa_hi, float *xa_lo, uint8_t *flags,
                                 void *workspace, int64_t workspace_bytes, void *stream)
{
    if (!delta) return lcs::set_error(LCS_E_ARG, "delta is NULL");
    if (!xa_hi || !xa_lo) return lcs::set_error(LCS_E_ARG, "xa_hi and xa_lo must not be NULL");
    return advect_sorted_impl(vel, seeds, 0, t0, T, dt, segment_steps, xa_hi, nullptr, flags,
                              workspace, workspace_bytes, stream, delta, xa_lo);
}

lcs_status lcs_advect_points(const lcs_velocity_t *vel, const float *x0, const double *t0, int64_t n,
                             double T, double dt, float *xf, int64_t *cell, uint8_t *flags,
                             void *stream)
{
    lcs_status st;
    if ((st = check_velocity(vel)) != LCS_OK) return st;
    if (!x0 || !t0 || !xf) return lcs::set_error(LCS_E_ARG, "x0, t0 and xf must not be NULL");
    if (n < 1 || n > kMaxSeeds) return lcs::set_error(LCS_E_SHAPE, "point count %lld out of range", (long long)n);
    int nsteps = 0;
    if ((st = check_steps(T, dt, &nsteps)) != LCS_OK) return st;
    lcs::AdvectArgs A;
    memset(&A, 0, sizeof(A));
    A.v = make_vel(vel);
    A.dt = dt;
    A.T = T;
    A.nsteps = nsteps;
    A.ns = n;
    A.x0 = x0;
    A.t0v = t0;
    A.xf = xf;
    A.cell = reinterpret_cast<long long *>(cell);
    A.flags = flags;
    hipError_t e = lcs::launch_advect_points(vel->dim, A, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "advect_points launch");
    return lcs::clear_error();
}

static lcs_status cg_common(const lcs_seed_grid_t *seeds, const float *xf, const uint8_t *flags,
                            lcs::CgArgs &A)
{
    lcs_status st;
    if (!seeds) return lcs::set_error(LCS_E_ARG, "seed grid descriptor is NULL");
    if ((st = check_seeds(seeds, seeds->dim)) != LCS_OK) return st;
    if (seeds->dim != 2 && seeds->dim != 3) return lcs::set_error(LCS_E_ARG, "seed dim must be 2 or 3");
    if (!xf) return lcs::set_error(LCS_E_ARG, "xf is NULL");
    if (seeds->n[1] > 65535 * 4 || seeds->n[2] > 65535)
        return lcs::set_error(LCS_E_SHAPE, "seed grid too tall for the launch shape");
    memset(&A, 0, sizeof(A));
    A.dim = seeds->dim;
    for (int a = 0; a < 3; ++a) {
        A.n[a] = (int)seeds->n[a];
        A.h[a] = seeds->spacing[a];
        A.period[a] = (double)seeds->n[a] * seeds->spacing[a];
    }
    A.periodic_mask = seeds->periodic_mask;
    A.ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    A.xf = xf;
    A.flags = flags;
    return LCS_OK;
}

lcs_status lcs_cg_tensor(const lcs_seed_grid_t *seeds, const float *xf, const uint8_t *flags,
                         double *C, uint8_t *stencil_flags, void *stream)
{
    lcs::CgArgs A;
    lcs_status st = cg_common(seeds, xf, flags, A);
    if (st != LCS_OK) return st;
    if (!C) return lcs::set_error(LCS_E_ARG, "C is NULL");
    A.C = C;
    A.sflags = stencil_flags;
    hipError_t e = lcs::launch_cg(A, false, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "cg launch");
    return lcs::clear_error();
}

lcs_status lcs_cg_ftle(const lcs_seed_grid_t *seeds, const float *xf, const uint8_t *flags, double T,
                       double *lambda_max, double *ftle, uint8_t *stencil_flags, void *stream)
{
    lcs::CgArgs A;
    lcs_status st = cg_common(seeds, xf, flags, A);
    if (st != LCS_OK) return st;
    if (!lambda_max && !ftle) return lcs::set_error(LCS_E_ARG, "lambda_max and ftle are both NULL");
    if (!isfinite(T) || T == 0.0) return lcs::set_error(LCS_E_ARG, "T must be finite and non-zero");
    A.lam = lambda_max;
    A.ftle = ftle;
    A.sflags = stencil_flags;
    A.inv_two_T = 1.0 / (2.0 * fabs(T));
    hipError_t e = lcs::launch_cg(A, true, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "cg_ftle launch");
    return lcs::clear_error();
}

lcs_status lcs_ftle(int32_t dim, int64_t n_points, const double *C, double T, double *lambda_max,
                    double *ftle, void *stream)
{
    if (dim != 2 && dim != 3) return lcs::set_error(LCS_E_ARG, "dim must be 2 or 3");
    if (n_points < 1 || n_points > kMaxSeeds) return lcs::set_error(LCS_E_SHAPE, "n_points out of range");
    if (!C) return lcs::set_error(LCS_E_ARG, "C is NULL");
    if (!lambda_max && !ftle) return lcs::set_error(LCS_E_ARG, "lambda_max and ftle are both NULL");
    if (!isfinite(T) || T == 0.0) return lcs::set_error(LCS_E_ARG, "T must be finite and non-zero");
    lcs::FtleArgs A;
    A.n = n_points;
    A.C = C;
    A.lam = lambda_max;
    A.ftle = ftle;
    A.inv_two_T = 1.0 / (2.0 * fabs(T));
    hipError_t e = lcs::launch_ftle(dim, A, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "ftle launch");
    return lcs::clear_error();
}

}  // extern "C"

extern "C" {

lcs_status lcs_advect_tuned(lcs_plan_t plan, const lcs_velocity_t *vel,
                            const lcs_seed_grid_t *seeds, double t0, double T, double dt,
                            float *xf, int64_t *cell, uint8_t *flags, void *workspace,
                            int64_t workspace_bytes, const int32_t *candidates,
                            int32_t n_candidates, int32_t *chosen, float *candidate_ms,
                            void *stream)
{
    if (!plan) return lcs::set_error(LCS_E_ARG, "plan is NULL");
    lcs_status st;
    if ((st = check_velocity(vel)) != LCS_OK) return st;
    if ((st = check_seeds(seeds, vel->dim)) != LCS_OK) return st;
    int nsteps = 0;
    if ((st = check_steps(T, dt, &nsteps)) != LCS_OK) return st;
    static const int32_t kDefault[] = {0, 200, 100, 50, 25};
    if (!candidates) {
        candidates = kDefault;
        n_candidates = 5;
    }
    if (n_candidates < 1 || n_candidates > 16)
        return lcs::set_error(LCS_E_ARG, "n_candidates must be 1..16");
    for (int i = 0; i < n_candidates; ++i)
        if (candidates[i] < 0) return lcs::set_error(LCS_E_ARG, "candidate segment lengths must be >= 0");
    int device = -1;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) return lcs::hip_error(e, "hipGetDevice");
    if (device != plan->device) return lcs::set_error(LCS_E_ARG, "plan belongs to device %d", plan->device);
    const bool ws_ok = workspace &&
                       workspace_bytes >= lcs_advect_sorted_workspace_bytes(vel, seeds);
    auto run = [&](int seg) {
        return seg == 0 ? lcs_advect(vel, seeds, t0, T, dt, xf, cell, flags, stream)
                        : lcs_advect_sorted(vel, seeds, t0, T, dt, seg, xf, cell, flags, workspace,
                                            workspace_bytes, stream);
    };
    const std::string key = tune_key(vel, seeds, nsteps, dt, device);
    for (auto &kv : plan->tuned) {
        if (kv.first != key) continue;
        const int seg = (kv.second != 0 && !ws_ok) ? 0 : kv.second;
        if (chosen) *chosen = seg;
        return run(seg);
    }
    // tune: one untimed run of the first eligible candidate, then each
    // eligible candidate once, timed with events on the caller's stream
    int first = -1;
    for (int i = 0; i < n_candidates && first < 0; ++i)
        if (candidates[i] == 0 || ws_ok) first = i;
    if (first < 0)
        return lcs::set_error(LCS_E_ARG, "no candidate can run: re-bundled candidates need a "
                              "workspace of lcs_advect_sorted_workspace_bytes");
    if ((st = run(candidates[first])) != LCS_OK) return st;
    hipEvent_t ev[2] = {nullptr, nullptr};
    e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    int best = -1;
    float best_ms = INFINITY;
    char msbuf[256] = "";
    for (int i = 0; i < n_candidates && e == hipSuccess; ++i) {
        const int seg = candidates[i];
        float ms = NAN;
        if (seg == 0 || ws_ok) {
            e = hipEventRecord(ev[0], (hipStream_t)stream);
            if (e != hipSuccess) break;
            if ((st = run(seg)) != LCS_OK) {
                (void)hipEventDestroy(ev[0]);
                (void)hipEventDestroy(ev[1]);
                return st;
            }
            e = hipEventRecord(ev[1], (hipStream_t)stream);
            if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (e == hipSuccess && ms < best_ms) {
                best_ms = ms;
                best = seg;
            }
        }
        if (candidate_ms) candidate_ms[i] = ms;
        const size_t used = strlen(msbuf);
        snprintf(msbuf + used, sizeof(msbuf) - used, "%s[%d, %.4g]", i ? ", " : "", seg,
                 isnan(ms) ? -1.0 : (double)ms);
    }
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    if (ev[1]) (void)hipEventDestroy(ev[1]);
    if (e != hipSuccess) return lcs::hip_error(e, "autotune timing");
    plan->tuned.emplace_back(key, best);
    if (!plan->cache_path.empty()) {
        FILE *f = fopen(plan->cache_path.c_str(), "a");
        if (f) {
            fprintf(f, "{\"key\": \"%s\", \"segment_steps\": %d, \"ms\": [%s]}\n", key.c_str(), best,
                    msbuf);
            fclose(f);
        }
    }
    if (chosen) *chosen = best;
    // every candidate computes the same bits, so the outputs of the last run
    // are the tuned call's outputs
    return lcs::clear_error();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// lcs_advect_sorted_noalloc: the re-bundled advection with its workspace in a
// fixed device array of this file instead of a caller buffer.  Each device
// that loads the library holds one copy (LCS_NOALLOC_SCRATCH_BYTES) until the
// process ends; its device address is looked up once per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[LCS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (host code must not pass
// the array's name itself to a kernel: on the host it is only a stand-in).
lcs_status scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return lcs::hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return lcs::set_error(LCS_E_UNSUPPORTED, "device %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return lcs::hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p) return lcs::set_error(LCS_E_HIP, "hipGetSymbolAddress(scratch) gave NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LCS_OK;
}
}  // namespace

extern "C" {

lcs_status lcs_advect_sorted_noalloc(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds,
                                     double t0, double T, double dt, int32_t segment_steps,
                                     float *xf, int64_t *cell, uint8_t *flags, void *stream)
{
    lcs_status st;
    if ((st = check_velocity(vel)) != LCS_OK) return st;
    if ((st = check_seeds(seeds, vel->dim)) != LCS_OK) return st;
    const long long n = seeds->n[0] * seeds->n[1] * seeds->n[2];
    const long long need = sorted_layout(vel, n, nullptr, nullptr).bytes;
    if (need > (long long)LCS_NOALLOC_SCRATCH_BYTES)
        return lcs::set_error(LCS_E_SHAPE, "this grid needs %lld bytes of scratch, more than the "
                              "%lld of lcs_advect_sorted_noalloc (use lcs_advect_sorted)",
                              need, (long long)LCS_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    if ((st = scratch_address(&ws)) != LCS_OK) return st;
    return advect_sorted_impl(vel, seeds, 0, t0, T, dt, segment_steps, xf, cell, flags, ws,
                              (int64_t)LCS_NOALLOC_SCRATCH_BYTES, stream);
}

}  // extern "C"
