/*
 * lcs_oracle.c -- plain, slow, FP64 CPU oracle for the LCS flow-map / FTLE path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * path (the HIP library) never links, calls or falls back to it, and the two
 * share no source, header, table or helper.
 *
 * What it computes (paper: Ameli, Desai & Shadden, "Development of an efficient
 * and flexible pipeline for Lagrangian coherent structure computation"):
 *
 *   - seed a structured grid of tracers                      (Sec. 2, Seed filter)
 *   - space-time interpolation of gridded velocity frames:
 *     multilinear in space, linear in time between the two
 *     frames that bracket t                                   (Sec. 2, Interpolator;
 *                                                              Sec. 3.2 grid kernels)
 *   - fixed-step classical RK4 integration of dx/dt = u(x,t)  (Eq. 2; Sec. 3.1)
 *   - trajectories that leave the domain are flagged and
 *     frozen at their last accepted position                  (Sec. 2, Flow Map filter)
 *   - flow-map gradient by central differences on the seed
 *     grid                                                     (Sec. 2, Cauchy-Green filter)
 *   - Cauchy-Green tensor C = grad(F)^T grad(F)                (Eq. 1)
 *   - largest eigenvalue of C and the FTLE                     (Sec. 1; Sec. 2)
 *
 * Readings where the paper is silent (each is stated where it is used):
 * node placement, the locate/tie-break rule, the domain-exit rule, one-sided
 * differences at non-periodic seed edges, the periodic-seam shift, and
 * FTLE = ln(lambda_max) / (2|T|).
 *
 * Everything is IEEE FP64, round-to-nearest, built with -ffp-contract=off.
 * Parallelism: independent tracers are distributed over OpenMP threads; no
 * tracer's arithmetic depends on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_FLAG_OUT 1u
#define ORC_FLAG_NONFINITE 2u
#define ORC_FLAG_STENCIL_OUT 4u
#define ORC_FLAG_TIME_OUT 8u

/* Velocity frames, structure of arrays: component c of node (i,j,k) in frame f
 * is u[c][f*n0*n1*n2 + i + n0*(j + n1*k)].  Node i of axis a is at
 * origin[a] + i*spacing[a].  A periodic axis a has period n[a]*spacing[a].
 * Frame f holds the field at t_first + f*dt_frame.  Frames stored in FP32
 * are read value by value and widened to FP64 (exact); all arithmetic is FP64. */
typedef struct {
    int32_t dim;
    int32_t n_frames;
    int64_t n[3];
    double origin[3];
    double spacing[3];
    uint32_t periodic_mask;
    uint32_t frames_f32;      /* 1: u[c] point to float arrays (widened on read) */
    double t_first;
    double dt_frame;
    const void *u[3];         /* double (or float if frames_f32) arrays */
} orc_velocity;

/* Structured seed grid: seed (i,j,k) at origin + (i,j,k)*spacing.  A periodic
 * seed axis has period n*spacing, which must equal the velocity period. */
typedef struct {
    int32_t dim;
    uint32_t periodic_mask;
    int64_t n[3];
    double origin[3];
    double spacing[3];
} orc_seed_grid;

static int axis_periodic(uint32_t mask, int a) { return (int)((mask >> a) & 1u); }

/* defined with the gradient and eigenvalue code below */
void orc_cg_point(const orc_seed_grid *g, const int64_t *ijk, const double *xc,
                  const double *const *xm, const double *const *xp, double *Cpacked);
double orc_lambda_max(int dim, const double *Cpacked);

/* ------------------------------------------------------------------------ */
/* Spatial location (reading: cell of a point along one axis)                */
/* ------------------------------------------------------------------------ */

/* Along axis a: s = (x - origin)/h in cell units.
 *  non-periodic: lower node i = floor(s), limited to [0, n-2]; a point on a
 *                face belongs to the higher cell except on the last face.
 *  periodic:     s is folded into [0, n) as s - n*floor(s/n); a fold that
 *                rounds up to exactly n is node 0; the upper node is (i+1) mod n.
 * Returns the lower node, the upper node and the local coordinate xi = s - i. */
static void locate_axis(double x, double origin, double h, int64_t n, int periodic,
                        int64_t *lo, int64_t *hi, double *xi)
{
    double s = (x - origin) / h;
    int64_t i;
    if (periodic) {
        double nd = (double)n;
        s = s - nd * floor(s / nd);
        i = (int64_t)floor(s);
        if (i >= n) { i = 0; s = 0.0; }
        if (i < 0) { i = 0; s = 0.0; }
        *lo = i;
        *hi = (i + 1 == n) ? 0 : i + 1;
    } else {
        i = (int64_t)floor(s);
        if (i > n - 2) i = n - 2;
        if (i < 0) i = 0;
        *lo = i;
        *hi = i + 1;
    }
    *xi = s - (double)i;
}

/* Linear index i + n0*(j + n1*k) of the lower corner of the velocity cell that
 * holds x (the rule of locate_axis).  Returns -1 for a non-finite point. */
int64_t orc_cell_index(const orc_velocity *v, const double *x)
{
    int64_t idx = 0, stride = 1;
    for (int a = 0; a < v->dim; ++a) {
        if (!isfinite(x[a])) return -1;
        int64_t lo, hi;
        double xi;
        locate_axis(x[a], v->origin[a], v->spacing[a], v->n[a],
                    axis_periodic(v->periodic_mask, a), &lo, &hi, &xi);
        idx += lo * stride;
        stride *= v->n[a];
    }
    return idx;
}

void orc_cell_index_many(const orc_velocity *v, const double *x, int64_t m, int64_t *cell)
{
    for (int64_t p = 0; p < m; ++p) {
        double q[3] = {0, 0, 0};
        for (int a = 0; a < v->dim; ++a) q[a] = x[a * m + p];
        cell[p] = orc_cell_index(v, q);
    }
}

/* Closed domain on non-periodic axes: origin <= x <= origin + (n-1)h.
 * Periodic axes never exit. */
int orc_in_domain(const orc_velocity *v, const double *x)
{
    for (int a = 0; a < v->dim; ++a) {
        if (axis_periodic(v->periodic_mask, a)) continue;
        double lo = v->origin[a];
        double hi = v->origin[a] + (double)(v->n[a] - 1) * v->spacing[a];
        if (!(x[a] >= lo && x[a] <= hi)) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Space-time interpolation                                                   */
/* ------------------------------------------------------------------------ */

static double node_value(const orc_velocity *v, int c, int64_t f, const int64_t idx[3])
{
    int64_t per_frame = v->n[0] * v->n[1] * v->n[2];
    int64_t lin = idx[0] + v->n[0] * (idx[1] + v->n[1] * idx[2]);
    if (v->frames_f32) return (double)((const float *)v->u[c])[f * per_frame + lin];
    return ((const double *)v->u[c])[f * per_frame + lin];
}

/* Multilinear interpolation of component c in frame f: the sum over the 2^dim
 * cell corners of the corner value times the product, over axes, of xi (upper
 * corner) or 1-xi (lower corner). */
static double frame_interp(const orc_velocity *v, int c, int64_t f,
                           const int64_t lo[3], const int64_t hi[3], const double xi[3])
{
    double acc = 0.0;
    int ncorner = 1 << v->dim;
    for (int corner = 0; corner < ncorner; ++corner) {
        double w = 1.0;
        int64_t idx[3] = {0, 0, 0};
        for (int a = 0; a < v->dim; ++a) {
            int upper = (corner >> a) & 1;
            idx[a] = upper ? hi[a] : lo[a];
            w *= upper ? xi[a] : (1.0 - xi[a]);
        }
        acc += w * node_value(v, c, f, idx);
    }
    return acc;
}

/* Frame pair bracketing t: f = floor((t - t_first)/dt_frame) limited to
 * [0, F-2]; alpha = (t - t_f)/dt_frame with t_f = t_first + f*dt_frame.
 * No extrapolation: callers keep t inside the frame span. */
static void frame_pair(const orc_velocity *v, double t, int64_t *f, double *alpha)
{
    double q = floor((t - v->t_first) / v->dt_frame);
    int64_t fi = (int64_t)q;
    if (fi > v->n_frames - 2) fi = v->n_frames - 2;
    if (fi < 0) fi = 0;
    double tf = v->t_first + (double)fi * v->dt_frame;
    *f = fi;
    *alpha = (t - tf) / v->dt_frame;
}

/* u(x, t): multilinear in space within each frame, then linear in time,
 * (1-alpha) u_f + alpha u_{f+1}.  x must be finite. */
void orc_velocity_at(const orc_velocity *v, const double *x, double t, double *out)
{
    int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    double xi[3] = {0, 0, 0};
    for (int a = 0; a < v->dim; ++a)
        locate_axis(x[a], v->origin[a], v->spacing[a], v->n[a],
                    axis_periodic(v->periodic_mask, a), &lo[a], &hi[a], &xi[a]);
    int64_t f;
    double alpha;
    frame_pair(v, t, &f, &alpha);
    for (int c = 0; c < v->dim; ++c) {
        double u0 = frame_interp(v, c, f, lo, hi, xi);
        double u1 = frame_interp(v, c, f + 1, lo, hi, xi);
        out[c] = (1.0 - alpha) * u0 + alpha * u1;
    }
}

void orc_velocity_at_many(const orc_velocity *v, const double *x, const double *t, int64_t m,
                          double *out)
{
    for (int64_t p = 0; p < m; ++p) {
        double q[3] = {0, 0, 0}, r[3] = {0, 0, 0};
        for (int a = 0; a < v->dim; ++a) q[a] = x[a * m + p];
        orc_velocity_at(v, q, t[p], r);
        for (int a = 0; a < v->dim; ++a) out[a * m + p] = r[a];
    }
}

/* ------------------------------------------------------------------------ */
/* RK4 advection                                                              */
/* ------------------------------------------------------------------------ */

static int all_finite(const double *x, int dim)
{
    for (int a = 0; a < dim; ++a)
        if (!isfinite(x[a])) return 0;
    return 1;
}

/* Check a point at which the field is about to be sampled (or a new
 * position): non-finite -> NONFINITE, outside the closed domain -> OUT. */
static uint32_t check_point(const orc_velocity *v, const double *p, double *margin)
{
    if (!all_finite(p, v->dim)) return ORC_FLAG_NONFINITE;
    if (margin) {
        /* diagnostic only: smallest distance, inside or outside, of a checked
         * point to a wall of the closed domain -- how close an in/out decision
         * came to going the other way */
        for (int a = 0; a < v->dim; ++a) {
            if (axis_periodic(v->periodic_mask, a)) continue;
            double lo = v->origin[a];
            double hi = v->origin[a] + (double)(v->n[a] - 1) * v->spacing[a];
            double d = fmin(fabs(p[a] - lo), fabs(hi - p[a]));
            if (d < *margin) *margin = d;
        }
    }
    if (!orc_in_domain(v, p)) return ORC_FLAG_OUT;
    return 0;
}

/* One classical RK4 step from (x, t) with step dt:
 *   k1 = u(x, t)
 *   k2 = u(x + dt/2 k1, t + dt/2)
 *   k3 = u(x + dt/2 k2, t + dt/2)
 *   k4 = u(x + dt k3,   t + dt)
 *   x' = x + dt/6 (k1 + 2 k2 + 2 k3 + k4)
 * Reading of the exit rule: if any stage point or x' is non-finite or outside
 * the closed domain (or a sampled velocity is non-finite), the step is
 * rejected, x is left unchanged and the matching flag is returned. */
static uint32_t rk4_step(const orc_velocity *v, double *x, double t, double dt, double *margin)
{
    int d = v->dim;
    double k1[3], k2[3], k3[3], k4[3], p[3], xn[3];
    uint32_t fl;

    orc_velocity_at(v, x, t, k1);
    if (!all_finite(k1, d)) return ORC_FLAG_NONFINITE;

    for (int a = 0; a < d; ++a) p[a] = x[a] + 0.5 * dt * k1[a];
    if ((fl = check_point(v, p, margin))) return fl;
    orc_velocity_at(v, p, t + 0.5 * dt, k2);
    if (!all_finite(k2, d)) return ORC_FLAG_NONFINITE;

    for (int a = 0; a < d; ++a) p[a] = x[a] + 0.5 * dt * k2[a];
    if ((fl = check_point(v, p, margin))) return fl;
    orc_velocity_at(v, p, t + 0.5 * dt, k3);
    if (!all_finite(k3, d)) return ORC_FLAG_NONFINITE;

    for (int a = 0; a < d; ++a) p[a] = x[a] + dt * k3[a];
    if ((fl = check_point(v, p, margin))) return fl;
    orc_velocity_at(v, p, t + dt, k4);
    if (!all_finite(k4, d)) return ORC_FLAG_NONFINITE;

    for (int a = 0; a < d; ++a)
        xn[a] = x[a] + (dt / 6.0) * (k1[a] + 2.0 * k2[a] + 2.0 * k3[a] + k4[a]);
    if ((fl = check_point(v, xn, margin))) return fl;

    for (int a = 0; a < d; ++a) x[a] = xn[a];
    return 0;
}

/* Integrate one tracer for nsteps fixed steps from t0: t_n = t0 + n*dt is
 * recomputed every step (never accumulated).  A rejected step freezes the
 * tracer and records its flag.  A starting point that is non-finite or
 * outside the domain is flagged before any step. */
static uint32_t advect_one(const orc_velocity *v, double *x, double t0, int64_t nsteps, double dt,
                           double *margin)
{
    uint32_t fl = check_point(v, x, margin);
    if (fl) return fl;
    for (int64_t n = 0; n < nsteps; ++n) {
        double t = t0 + (double)n * dt;
        fl = rk4_step(v, x, t, dt, margin);
        if (fl) return fl;
    }
    return 0;
}

/* No extrapolation in time (the paper cautions against extrapolating the
 * velocity, Sec. 2 Flow Map filter): a point whose interval [t0, t0+T] is not
 * inside the frame span [t_first, t_first + (F-1) dt_frame] is not advected
 * and is flagged TIME_OUT. */
static int time_span_ok(const orc_velocity *v, double t0, double T)
{
    double t_last = v->t_first + (double)(v->n_frames - 1) * v->dt_frame;
    double t1 = t0 + T;
    return t0 >= v->t_first && t0 <= t_last && t1 >= v->t_first && t1 <= t_last;
}

/* Number of fixed steps: N = round(T/dt).  The caller has checked that T/dt
 * is integral. */
static int64_t step_count(double T, double dt) { return (int64_t)llround(T / dt); }

/* Advect arbitrary points x0 (dim x m, SoA), each from its own t0[p], over
 * the same duration T with step dt.  Outputs (any may be NULL): xf (dim x m),
 * cell (m), flags (m), margin (m): the smallest distance, inside or outside,
 * of any checked stage point or position to a wall of the closed domain (a
 * diagnostic used to tell which tracers came too close to a wall for an FP32
 * run to take the same in/out decisions). */
void orc_advect_points(const orc_velocity *v, const double *x0, const double *t0, int64_t m,
                       double T, double dt, double *xf, int64_t *cell, uint8_t *flags,
                       double *margin, int nthreads)
{
    int64_t nsteps = step_count(T, dt);
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t p = 0; p < m; ++p) {
        double x[3] = {0, 0, 0};
        for (int a = 0; a < v->dim; ++a) x[a] = x0[a * m + p];
        double mg = INFINITY;
        uint32_t fl = time_span_ok(v, t0[p], T) ? advect_one(v, x, t0[p], nsteps, dt, &mg)
                                                : ORC_FLAG_TIME_OUT;
        if (margin) margin[p] = mg;
        if (xf)
            for (int a = 0; a < v->dim; ++a) xf[a * m + p] = x[a];
        if (cell) cell[p] = orc_cell_index(v, x);
        if (flags) flags[p] = (uint8_t)fl;
    }
    (void)nthreads;
}

/* Seed positions of the structured grid (step "Seed"): seed with integer
 * coordinates (i,j,k) sits at origin + (i,j,k)*spacing, computed in FP64. */
static void seed_position(const orc_seed_grid *g, int64_t lin, double *x)
{
    int64_t i = lin % g->n[0];
    int64_t r = lin / g->n[0];
    int64_t j = r % g->n[1];
    int64_t k = r / g->n[1];
    int64_t ijk[3] = {i, j, k};
    for (int a = 0; a < g->dim; ++a) x[a] = g->origin[a] + (double)ijk[a] * g->spacing[a];
}

void orc_seed_points(const orc_seed_grid *g, const int64_t *idx, int64_t m, double *x)
{
    for (int64_t p = 0; p < m; ++p) {
        double q[3] = {0, 0, 0};
        seed_position(g, idx[p], q);
        for (int a = 0; a < g->dim; ++a) x[a * m + p] = q[a];
    }
}

/* Advect the seeds with the given linear indices (all seeds if idx == NULL,
 * then m must be the seed count) from one t0.  Output arrays are indexed like
 * idx: xf is dim x m. */
void orc_advect_seeds(const orc_velocity *v, const orc_seed_grid *g, const int64_t *idx, int64_t m,
                      double t0, double T, double dt, double *xf, int64_t *cell, uint8_t *flags,
                      double *margin, int nthreads)
{
    int64_t nsteps = step_count(T, dt);
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t p = 0; p < m; ++p) {
        double x[3] = {0, 0, 0};
        seed_position(g, idx ? idx[p] : p, x);
        double mg = INFINITY;
        uint32_t fl = advect_one(v, x, t0, nsteps, dt, &mg);
        if (margin) margin[p] = mg;
        if (xf)
            for (int a = 0; a < v->dim; ++a) xf[a * m + p] = x[a];
        if (cell) cell[p] = orc_cell_index(v, x);
        if (flags) flags[p] = (uint8_t)fl;
    }
    (void)nthreads;
}

/* ------------------------------------------------------------------------ */
/* Time-resolved and early Cauchy-Green evaluation                            */
/* ------------------------------------------------------------------------ */

/* Flow map at several integration times (Sec. 3.1: the CG tensor can be
 * evaluated at any step of the interval; Sec. 4: CG fields wanted at several
 * instants).  snap_steps (n_snap values, strictly increasing, >= 1): the step
 * counts at which positions are recorded; xf[(k*dim + a)*m + p] and
 * flags[k*m + p] hold snapshot k (a tracer frozen earlier keeps its frozen
 * position and its flag); steps_done[p] = accepted steps before the tracer
 * froze (the last snapshot's step count if it never did). */
void orc_advect_seeds_snap(const orc_velocity *v, const orc_seed_grid *g, const int64_t *idx,
                           int64_t m, double t0, double dt, int n_snap, const int64_t *snap_steps,
                           double *xf, uint8_t *flags, int64_t *steps_done, int nthreads)
{
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t p = 0; p < m; ++p) {
        double x[3] = {0, 0, 0};
        seed_position(g, idx ? idx[p] : p, x);
        uint32_t fl = check_point(v, x, NULL);
        int64_t nacc = 0;
        int k = 0;
        int64_t last = snap_steps[n_snap - 1];
        for (int64_t n = 0; n < last; ++n) {
            if (!fl) {
                fl = rk4_step(v, x, t0 + (double)n * dt, dt, NULL);
                if (!fl) nacc = n + 1;
            }
            if (n + 1 == snap_steps[k]) {
                for (int a = 0; a < v->dim; ++a) xf[((int64_t)k * v->dim + a) * m + p] = x[a];
                flags[(int64_t)k * m + p] = (uint8_t)fl;
                ++k;
            }
        }
        if (steps_done) steps_done[p] = nacc;
    }
    (void)nthreads;
}

/* Seeds whose final positions the gradient at seed (ijk) uses (the seed itself
 * and its lower/upper neighbours along each axis, as orc_cg_point differences
 * them); returns their count and writes their linear indices. */
static int stencil_members(const orc_seed_grid *g, const int64_t *ijk, int64_t *out)
{
    int k = 0;
    out[k++] = ijk[0] + g->n[0] * (ijk[1] + g->n[1] * ijk[2]);
    for (int b = 0; b < g->dim; ++b) {
        int64_t n = g->n[b];
        int per = axis_periodic(g->periodic_mask, b);
        for (int dir = -1; dir <= 1; dir += 2) {
            int64_t c[3] = {ijk[0], ijk[1], ijk[2]};
            int64_t j = c[b] + dir;
            if (per) j = (j + n) % n;
            else if (j < 0 || j >= n) continue;   /* one-sided: the seed itself */
            c[b] = j;
            out[k++] = c[0] + g->n[0] * (c[1] + g->n[1] * c[2]);
        }
    }
    return k;
}

/* Early evaluation (Sec. 2 Flow Map filter: when a trajectory leaves the
 * domain, the CG tensor is evaluated early at every location that relies on
 * it).  Reading: for seed s, n_s = the smallest steps_done over the seeds its
 * gradient uses; its members are advected n_s steps from t0, C is formed from
 * those positions by orc_cg_point and sigma = ln(lambda_max) / (2 n_s |dt|),
 * t_eff = n_s dt.  n_s = 0 gives NaN.  For seeds whose stencil never left,
 * n_s = nsteps and the result is the ordinary FTLE.  Outputs for the seeds
 * idx (all if NULL, m = seed count); lam, ftle, t_eff may be NULL. */
void orc_ftle_early(const orc_velocity *v, const orc_seed_grid *g, const int64_t *idx, int64_t m,
                    double t0, double dt, const int64_t *steps_done, double *lam, double *ftle,
                    double *t_eff, int nthreads)
{
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
#endif
    for (int64_t p = 0; p < m; ++p) {
        int64_t s = idx ? idx[p] : p;
        int64_t ijk[3] = {s % g->n[0], (s / g->n[0]) % g->n[1], s / (g->n[0] * g->n[1])};
        int64_t mem[7];
        int nm = stencil_members(g, ijk, mem);
        int64_t ns = steps_done[mem[0]];
        for (int q = 1; q < nm; ++q)
            if (steps_done[mem[q]] < ns) ns = steps_done[mem[q]];
        double l = NAN, f = NAN;
        if (ns > 0) {
            /* positions of the seed and its neighbours after ns steps */
            double xc[3] = {0, 0, 0}, xmv[3][3], xpv[3][3];
            const double *xm[3], *xp[3];
            seed_position(g, s, xc);
            advect_one(v, xc, t0, ns, dt, NULL);
            for (int b = 0; b < g->dim; ++b) {
                for (int side = 0; side < 2; ++side) {
                    int64_t c[3] = {ijk[0], ijk[1], ijk[2]};
                    int64_t n = g->n[b];
                    int64_t j = c[b] + (side ? 1 : -1);
                    double *dst = side ? xpv[b] : xmv[b];
                    if (axis_periodic(g->periodic_mask, b)) j = (j + n) % n;
                    if (j < 0 || j >= n) {          /* unused by the one-sided formula */
                        for (int a = 0; a < 3; ++a) dst[a] = xc[a];
                        continue;
                    }
                    c[b] = j;
                    double x[3] = {0, 0, 0};
                    seed_position(g, c[0] + g->n[0] * (c[1] + g->n[1] * c[2]), x);
                    advect_one(v, x, t0, ns, dt, NULL);
                    for (int a = 0; a < 3; ++a) dst[a] = x[a];
                }
                xm[b] = xmv[b];
                xp[b] = xpv[b];
            }
            double C[6];
            orc_cg_point(g, ijk, xc, xm, xp, C);
            l = orc_lambda_max(g->dim, C);
            f = (l > 0.0) ? log(l) / (2.0 * fabs((double)ns * dt)) : -INFINITY;
        }
        if (lam) lam[p] = l;
        if (ftle) ftle[p] = f;
        if (t_eff) t_eff[p] = (double)ns * dt;
    }
    (void)nthreads;
}

/* ------------------------------------------------------------------------ */
/* Auxiliary points                                                           */
/* ------------------------------------------------------------------------ */

/* Auxiliary points about each seed (Sec. 2 Seed filter) for the flow-map
 * gradient (Sec. 2 Cauchy-Green filter): around seed x0, for every axis b < dim
 * one point at x0 - delta_b e_b (side 0) and one at x0 + delta_b e_b (side 1).
 * Output x is dim x (2 dim m): component a of auxiliary point q = 2b + side of
 * the p-th listed seed at x[a*(2 dim m) + q*m + p]. */
void orc_aux_points(const orc_seed_grid *g, const int64_t *idx, int64_t m, const double *delta,
                    double *x)
{
    int d = g->dim;
    int64_t w = 2 * (int64_t)d * m;
    for (int64_t p = 0; p < m; ++p) {
        double x0[3] = {0, 0, 0};
        seed_position(g, idx ? idx[p] : p, x0);
        for (int b = 0; b < d; ++b)
            for (int side = 0; side < 2; ++side) {
                int64_t q = 2 * b + side;
                for (int a = 0; a < d; ++a) {
                    double v = x0[a];
                    if (a == b) v = side ? x0[a] + delta[b] : x0[a] - delta[b];
                    x[a * w + q * m + p] = v;
                }
            }
    }
}

/* Flow-map gradient from the final positions of the auxiliary points:
 *   J[a][b] = (F_a(x0 + delta_b e_b) - F_a(x0 - delta_b e_b)) / (2 delta_b),
 * C = J^T J packed as orc_cg_point.  xf is laid out as orc_aux_points' x;
 * flags (2 dim m, or NULL) are the auxiliary tracers' flags, and a seed whose
 * auxiliary points include a flagged one gets STENCIL_OUT. */
void orc_cg_aux(int dim, int64_t m, const double *delta, const double *xf, const uint8_t *flags,
                double *C, uint8_t *sflags)
{
    int64_t w = 2 * (int64_t)dim * m;
    int nq = dim * (dim + 1) / 2;
    for (int64_t p = 0; p < m; ++p) {
        double J[3][3] = {{0}};
        uint8_t bad = 0;
        for (int b = 0; b < dim; ++b) {
            int64_t qm = 2 * b, qp = 2 * b + 1;
            for (int a = 0; a < dim; ++a)
                J[a][b] = (xf[a * w + qp * m + p] - xf[a * w + qm * m + p]) / (2.0 * delta[b]);
            if (flags && (flags[qm * m + p] || flags[qp * m + p])) bad = 1;
        }
        int k = 0;
        for (int r = 0; r < dim; ++r)
            for (int s = r; s < dim; ++s) {
                double acc = 0.0;
                for (int a = 0; a < dim; ++a) acc += J[a][r] * J[a][s];
                C[(int64_t)k++ * m + p] = acc;
            }
        (void)nq;
        if (sflags) sflags[p] = bad ? ORC_FLAG_STENCIL_OUT : 0;
    }
}

/* ------------------------------------------------------------------------ */
/* Adams-Bashforth multistep integration                                      */
/* ------------------------------------------------------------------------ */

/* The Flow Map filter admits multistep methods such as Adams-Bashforth
 * (Sec. 2).  Explicit s-step Adams-Bashforth, s = 2, 3 or 4:
 *   x_{n+1} = x_n + dt * sum_{j=0}^{s-1} b_j f_{n-j},   f_m = u(x_m, t_m),
 * with the classical coefficients b = (3, -1)/2, (23, -16, 5)/12 and
 * (55, -59, 37, -9)/24.  Readings (the paper names the family only): the
 * first s-1 steps are classical RK4 steps, whose first-stage values are the
 * f_m of those steps; the exit rule is the RK4 one applied to the one new
 * point of a multistep step, x_{n+1}. */
static double ab_coef(int order, int j)
{
    if (order == 2) {
        const double b[2] = {3.0 / 2.0, -1.0 / 2.0};
        return b[j];
    }
    if (order == 3) {
        const double b[3] = {23.0 / 12.0, -16.0 / 12.0, 5.0 / 12.0};
        return b[j];
    }
    const double b[4] = {55.0 / 24.0, -59.0 / 24.0, 37.0 / 24.0, -9.0 / 24.0};
    return b[j];
}

static uint32_t advect_one_ab(const orc_velocity *v, double *x, double t0, int64_t nsteps,
                              double dt, int order, double *margin)
{
    uint32_t fl = check_point(v, x, margin);
    if (fl) return fl;
    int d = v->dim;
    double hist[4][3] = {{0}};   /* hist[j] = f_{n-j} */
    for (int64_t n = 0; n < nsteps; ++n) {
        double t = t0 + (double)n * dt;
        double f[3];
        orc_velocity_at(v, x, t, f);
        if (!all_finite(f, d)) return ORC_FLAG_NONFINITE;
        for (int j = 3; j > 0; --j)
            for (int a = 0; a < d; ++a) hist[j][a] = hist[j - 1][a];
        for (int a = 0; a < d; ++a) hist[0][a] = f[a];
        if (n < order - 1) {
            fl = rk4_step(v, x, t, dt, margin);
            if (fl) return fl;
            continue;
        }
        double xn[3];
        for (int a = 0; a < d; ++a) {
            double s = 0.0;
            for (int j = 0; j < order; ++j) s += ab_coef(order, j) * hist[j][a];
            xn[a] = x[a] + dt * s;
        }
        if ((fl = check_point(v, xn, margin))) return fl;
        for (int a = 0; a < d; ++a) x[a] = xn[a];
    }
    return 0;
}

/* Adams-Bashforth flow map of the seed grid (or the seeds idx): outputs as
 * for orc_advect_seeds. */
void orc_advect_seeds_ab(const orc_velocity *v, const orc_seed_grid *g, const int64_t *idx,
                         int64_t m, double t0, double T, double dt, int order, double *xf,
                         int64_t *cell, uint8_t *flags, double *margin, int nthreads)
{
    int64_t nsteps = step_count(T, dt);
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t p = 0; p < m; ++p) {
        double x[3] = {0, 0, 0};
        seed_position(g, idx ? idx[p] : p, x);
        double mg = INFINITY;
        uint32_t fl = advect_one_ab(v, x, t0, nsteps, dt, order, &mg);
        if (margin) margin[p] = mg;
        if (xf)
            for (int a = 0; a < v->dim; ++a) xf[a * m + p] = x[a];
        if (cell) cell[p] = orc_cell_index(v, x);
        if (flags) flags[p] = (uint8_t)fl;
    }
    (void)nthreads;
}

/* Adams-Bashforth flow map of arbitrary points, each from its own t0. */
void orc_advect_points_ab(const orc_velocity *v, const double *x0, const double *t0, int64_t m,
                          double T, double dt, int order, double *xf, int64_t *cell,
                          uint8_t *flags, double *margin, int nthreads)
{
    int64_t nsteps = step_count(T, dt);
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t p = 0; p < m; ++p) {
        double x[3] = {0, 0, 0};
        for (int a = 0; a < v->dim; ++a) x[a] = x0[a * m + p];
        double mg = INFINITY;
        uint32_t fl = time_span_ok(v, t0[p], T) ? advect_one_ab(v, x, t0[p], nsteps, dt, order, &mg)
                                                : ORC_FLAG_TIME_OUT;
        if (margin) margin[p] = mg;
        if (xf)
            for (int a = 0; a < v->dim; ++a) xf[a * m + p] = x[a];
        if (cell) cell[p] = orc_cell_index(v, x);
        if (flags) flags[p] = (uint8_t)fl;
    }
    (void)nthreads;
}

/* Trajectory recording for the mean-trajectory-error curves (Sec. 3.3): the
 * positions of every point after each of the N steps, traj[(n*dim + a)*m + p]. */
void orc_advect_points_traj(const orc_velocity *v, const double *x0, const double *t0, int64_t m,
                            double T, double dt, double *traj, uint8_t *flags, int nthreads)
{
    int64_t nsteps = step_count(T, dt);
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t p = 0; p < m; ++p) {
        double x[3] = {0, 0, 0};
        for (int a = 0; a < v->dim; ++a) x[a] = x0[a * m + p];
        uint32_t fl = time_span_ok(v, t0[p], T) ? check_point(v, x, NULL) : ORC_FLAG_TIME_OUT;
        for (int64_t n = 0; n < nsteps; ++n) {
            if (!fl) fl = rk4_step(v, x, t0[p] + (double)n * dt, dt, NULL);
            for (int a = 0; a < v->dim; ++a) traj[(n * v->dim + a) * m + p] = x[a];
        }
        if (flags) flags[p] = (uint8_t)fl;
    }
    (void)nthreads;
}

/* ------------------------------------------------------------------------ */
/* Flow-map gradient and Cauchy-Green tensor                                  */
/* ------------------------------------------------------------------------ */

/* Gradient of the flow map at one seed with integer coordinates ijk, from the
 * final positions of the seed (xc) and of its lower and upper neighbours
 * along each axis b (xm[b], xp[b]); each is a dim-vector.
 *   interior (and every periodic axis):  J[a][b] = (F_a(+) - F_a(-)) / (2 h_b)
 *   non-periodic first seed (i = 0):     J[a][b] = (F_a(i+1) - F_a(i)) / h_b
 *   non-periodic last seed (i = n-1):    J[a][b] = (F_a(i) - F_a(i-1)) / h_b
 * (one-sided first-order differences at edges are the reading; the paper
 * only names central differences).  On a periodic axis the neighbour across
 * the seam is the seed on the far side, and its component b is shifted by the
 * period L_b = n_b h_b: F(x0 + L e_b) = F(x0) + L e_b for a periodic field.
 * Then C = J^T J, packed (xx, xy, yy) in 2D or (xx, xy, xz, yy, yz, zz) in 3D. */
void orc_cg_point(const orc_seed_grid *g, const int64_t *ijk, const double *xc,
                  const double *const *xm, const double *const *xp, double *Cpacked)
{
    int d = g->dim;
    double J[3][3] = {{0}};
    for (int b = 0; b < d; ++b) {
        int64_t i = ijk[b], n = g->n[b];
        double h = g->spacing[b];
        if (axis_periodic(g->periodic_mask, b)) {
            double L = (double)n * h;
            double shift_p = (i + 1 >= n) ? L : 0.0;
            double shift_m = (i - 1 < 0) ? -L : 0.0;
            for (int a = 0; a < d; ++a) {
                double fp = xp[b][a] + (a == b ? shift_p : 0.0);
                double fm = xm[b][a] + (a == b ? shift_m : 0.0);
                J[a][b] = (fp - fm) / (2.0 * h);
            }
        } else if (i == 0) {
            for (int a = 0; a < d; ++a) J[a][b] = (xp[b][a] - xc[a]) / h;
        } else if (i == n - 1) {
            for (int a = 0; a < d; ++a) J[a][b] = (xc[a] - xm[b][a]) / h;
        } else {
            for (int a = 0; a < d; ++a) J[a][b] = (xp[b][a] - xm[b][a]) / (2.0 * h);
        }
    }
    int k = 0;
    for (int r = 0; r < d; ++r)
        for (int s = r; s < d; ++s) {
            double acc = 0.0;
            for (int a = 0; a < d; ++a) acc += J[a][r] * J[a][s];
            Cpacked[k++] = acc;
        }
}

/* Neighbour index along axis b: wraps on periodic axes, clamps (and is then
 * unused or equal to the seed) on non-periodic ones. */
static int64_t neighbour(const orc_seed_grid *g, int b, int64_t i, int dir)
{
    int64_t n = g->n[b];
    int64_t j = i + dir;
    if (axis_periodic(g->periodic_mask, b)) {
        if (j < 0) j += n;
        if (j >= n) j -= n;
    } else {
        if (j < 0) j = 0;
        if (j >= n) j = n - 1;
    }
    return j;
}

/* C on the whole seed grid from final positions xf (dim x Ns).  flags (may be
 * NULL) marks tracers that left the domain or met non-finite data; every seed
 * whose stencil (itself and the neighbours it differences) holds a flagged
 * tracer gets STENCIL_OUT in sflags.  C is packed SoA: C[q*Ns + s]. */
void orc_cg_tensor(const orc_seed_grid *g, const double *xf, const uint8_t *flags, double *C,
                   uint8_t *sflags, int nthreads)
{
    int d = g->dim;
    int64_t Ns = g->n[0] * g->n[1] * g->n[2];
    int nq = d * (d + 1) / 2;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int64_t s = 0; s < Ns; ++s) {
        int64_t ijk[3] = {s % g->n[0], (s / g->n[0]) % g->n[1], s / (g->n[0] * g->n[1])};
        int64_t stride[3] = {1, g->n[0], g->n[0] * g->n[1]};
        double xc[3], xmv[3][3], xpv[3][3];
        const double *xm[3], *xp[3];
        uint8_t any = flags ? flags[s] : 0;
        for (int a = 0; a < d; ++a) xc[a] = xf[a * Ns + s];
        for (int b = 0; b < d; ++b) {
            int64_t im = neighbour(g, b, ijk[b], -1), ip = neighbour(g, b, ijk[b], +1);
            int64_t sm = s + (im - ijk[b]) * stride[b];
            int64_t sp = s + (ip - ijk[b]) * stride[b];
            for (int a = 0; a < d; ++a) {
                xmv[b][a] = xf[a * Ns + sm];
                xpv[b][a] = xf[a * Ns + sp];
            }
            xm[b] = xmv[b];
            xp[b] = xpv[b];
            if (flags) any |= flags[sm] | flags[sp];
        }
        double Cp[6];
        orc_cg_point(g, ijk, xc, xm, xp, Cp);
        for (int q = 0; q < nq; ++q) C[q * Ns + s] = Cp[q];
        if (sflags) sflags[s] = any ? ORC_FLAG_STENCIL_OUT : 0;
    }
    (void)nthreads;
}

/* ------------------------------------------------------------------------ */
/* Largest eigenvalue and FTLE                                                */
/* ------------------------------------------------------------------------ */

/* 2x2 symmetric [[a, b], [b, c]]: lambda_max = (a+c)/2 + sqrt(((a-c)/2)^2 + b^2). */
static double eig_max_sym2(const double *c)
{
    double a = c[0], b = c[1], d = c[2];
    return 0.5 * (a + d) + hypot(0.5 * (a - d), b);
}

/* 3x3 symmetric: cyclic Jacobi.  Each rotation J(p,q,theta) is chosen so that
 * (J^T A J)[p][q] = 0 (Golub & Van Loan, symmetric Schur decomposition); the
 * product J^T A J is formed explicitly.  Sweeps stop when the off-diagonal
 * mass is negligible against the diagonal; lambda_max is the largest diagonal
 * entry. */
static double eig_max_sym3(const double *c)
{
    double A[3][3] = {{c[0], c[1], c[2]}, {c[1], c[3], c[4]}, {c[2], c[4], c[5]}};
    static const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off == 0.0 || off <= 1e-36 * dia) break;
        for (int r = 0; r < 3; ++r) {
            int p = pairs[r][0], q = pairs[r][1];
            if (A[p][q] == 0.0) continue;
            double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
            double t = (tau >= 0.0) ? 1.0 / (tau + hypot(1.0, tau))
                                    : 1.0 / (tau - hypot(1.0, tau));
            double cs = 1.0 / sqrt(1.0 + t * t);
            double sn = t * cs;
            double R[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
            R[p][p] = cs;
            R[q][q] = cs;
            R[p][q] = sn;
            R[q][p] = -sn;
            double T1[3][3], B[3][3];
            for (int i = 0; i < 3; ++i)          /* T1 = A R */
                for (int j = 0; j < 3; ++j) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; ++k) acc += A[i][k] * R[k][j];
                    T1[i][j] = acc;
                }
            for (int i = 0; i < 3; ++i)          /* B = R^T T1 */
                for (int j = 0; j < 3; ++j) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; ++k) acc += R[k][i] * T1[k][j];
                    B[i][j] = acc;
                }
            for (int i = 0; i < 3; ++i)          /* keep exact symmetry */
                for (int j = 0; j < 3; ++j) A[i][j] = (i <= j) ? B[i][j] : B[j][i];
            A[p][q] = A[q][p] = 0.0;
        }
    }
    double m = A[0][0];
    if (A[1][1] > m) m = A[1][1];
    if (A[2][2] > m) m = A[2][2];
    return m;
}

double orc_lambda_max(int dim, const double *Cpacked)
{
    return dim == 2 ? eig_max_sym2(Cpacked) : eig_max_sym3(Cpacked);
}

/* Eigenvalues and eigenvectors of the symmetric C (Sec. 2 Cauchy-Green filter:
 * eigenvalue/eigenvector fields for LCS detection).  Cyclic Jacobi on the
 * dim x dim matrix with the rotations accumulated, V <- V R, each product formed
 * explicitly; then the pairs are sorted by ascending eigenvalue and every
 * eigenvector is normalised in sign so that its component of largest magnitude
 * (the first such on a tie) is positive -- the reading that makes the otherwise
 * sign-free eigenvectors comparable.  evals[k], evecs[k*dim + a] = component a
 * of eigenvector k. */
void orc_eig_sym(int dim, const double *c, double *evals, double *evecs)
{
    double A[3][3] = {{0}}, V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    int k = 0;
    for (int i = 0; i < dim; ++i)
        for (int j = i; j < dim; ++j) A[i][j] = A[j][i] = c[k++];
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int i = 0; i < dim; ++i) {
            dia += A[i][i] * A[i][i];
            for (int j = i + 1; j < dim; ++j) off += A[i][j] * A[i][j];
        }
        if (off == 0.0 || off <= 1e-36 * dia) break;
        for (int p = 0; p < dim; ++p)
            for (int q = p + 1; q < dim; ++q) {
                if (A[p][q] == 0.0) continue;
                double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (tau >= 0.0) ? 1.0 / (tau + hypot(1.0, tau))
                                        : 1.0 / (tau - hypot(1.0, tau));
                double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
                double R[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
                R[p][p] = cs;
                R[q][q] = cs;
                R[p][q] = sn;
                R[q][p] = -sn;
                double T1[3][3], B[3][3], W[3][3];
                for (int i = 0; i < dim; ++i)
                    for (int j = 0; j < dim; ++j) {
                        double a1 = 0.0, a2 = 0.0;
                        for (int m = 0; m < dim; ++m) {
                            a1 += A[i][m] * R[m][j];
                            a2 += V[i][m] * R[m][j];
                        }
                        T1[i][j] = a1;
                        W[i][j] = a2;
                    }
                for (int i = 0; i < dim; ++i)
                    for (int j = 0; j < dim; ++j) {
                        double acc = 0.0;
                        for (int m = 0; m < dim; ++m) acc += R[m][i] * T1[m][j];
                        B[i][j] = acc;
                    }
                for (int i = 0; i < dim; ++i)
                    for (int j = 0; j < dim; ++j) {
                        A[i][j] = (i <= j) ? B[i][j] : B[j][i];
                        V[i][j] = W[i][j];
                    }
                A[p][q] = A[q][p] = 0.0;
            }
    }
    int order[3] = {0, 1, 2};
    for (int i = 0; i < dim; ++i)          /* ascending eigenvalues (stable) */
        for (int j = i + 1; j < dim; ++j)
            if (A[order[j]][order[j]] < A[order[i]][order[i]]) {
                int t = order[i];
                order[i] = order[j];
                order[j] = t;
            }
    for (int e = 0; e < dim; ++e) {
        int col = order[e];
        evals[e] = A[col][col];
        int big = 0;
        for (int a = 1; a < dim; ++a)
            if (fabs(V[a][col]) > fabs(V[big][col])) big = a;
        double sgn = (V[big][col] < 0.0) ? -1.0 : 1.0;
        for (int a = 0; a < dim; ++a) evecs[e * dim + a] = sgn * V[a][col];
    }
}

/* orc_eig_sym over n packed tensors (nq x n): evals[k*n + p],
 * evecs[(k*dim + a)*n + p]. */
void orc_eig_many(int dim, int64_t n, const double *C, double *evals, double *evecs)
{
    int nq = dim * (dim + 1) / 2;
    for (int64_t p = 0; p < n; ++p) {
        double c[6], ev[3], V[9];
        for (int q = 0; q < nq; ++q) c[q] = C[q * n + p];
        orc_eig_sym(dim, c, ev, V);
        for (int k = 0; k < dim; ++k) {
            evals[k * n + p] = ev[k];
            for (int a = 0; a < dim; ++a) evecs[(k * dim + a) * n + p] = V[k * dim + a];
        }
    }
}

/* FTLE (reading: the standard definition of the cited FTLE work)
 *   sigma = ln(lambda_max) / (2 |T|);  lambda_max <= 0 (only if grad F = 0)
 * gives -inf.  C is packed SoA with Ns points; lam and ftle may be NULL. */
void orc_ftle(int dim, int64_t Ns, const double *C, double T, double *lam, double *ftle,
              int nthreads)
{
    int nq = dim * (dim + 1) / 2;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int64_t s = 0; s < Ns; ++s) {
        double c[6];
        for (int q = 0; q < nq; ++q) c[q] = C[q * Ns + s];
        double l = orc_lambda_max(dim, c);
        if (lam) lam[s] = l;
        if (ftle) ftle[s] = (l > 0.0) ? log(l) / (2.0 * fabs(T)) : -INFINITY;
    }
    (void)nthreads;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ======================================================================== */
/* Unstructured meshes: triangles (2D) and tetrahedra (3D)                    */
/* ======================================================================== */
/*
 * Velocity given at the nodes of a conforming triangle or tetrahedron mesh
 * (Sec. 3.2: unstructured data is tetrahedralised so that one cell search and
 * one interpolation serve every grid topology).  Inside a cell the field is
 * the piecewise-linear interpolant u(x) = sum_i lambda_i(x) u(node_i), lambda
 * the barycentric coordinates of x in that cell; in time it is linear between
 * the two frames that bracket t, as on structured grids.
 *
 * The oracle finds the cell holding a point with a structured auxiliary grid
 * of buckets over the mesh's bounding box, each bucket listing every cell
 * whose bounding box meets it, and tests the listed cells; it does not use
 * the local neighbour walk of the GPU code.  The interpolant does not depend
 * on how the cell is found (it is continuous across faces).
 */
typedef struct {
    int32_t dim;
    int32_t n_frames;
    int64_t n_nodes;
    int64_t n_cells;
    const double *nodes;   /* [n_nodes][dim] */
    const int32_t *cells;  /* [n_cells][dim+1] */
    double t_first;
    double dt_frame;
    const double *u;       /* [n_frames][n_nodes][dim] */
    double lo[3], hi[3];   /* bounding box of the nodes */
    double bsize[3];
    int64_t nb[3];
    int64_t *bstart;       /* CSR offsets, nb[0]*nb[1]*nb[2] + 1 */
    int32_t *bcells;
    double tol;            /* a point is in a cell if every lambda >= -tol */
} orc_mesh;

/* (b - a) x (c - a): twice the signed area of triangle abc */
static double area2(const double *a, const double *b, const double *c)
{
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

/* (b - a) . ((c - a) x (d - a)): six times the signed volume of tetrahedron abcd */
static double vol6(const double *a, const double *b, const double *c, const double *d)
{
    double e1[3], e2[3], e3[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = b[k] - a[k];
        e2[k] = c[k] - a[k];
        e3[k] = d[k] - a[k];
    }
    return e1[0] * (e2[1] * e3[2] - e2[2] * e3[1])
         - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0])
         + e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
}

static const double *mesh_node(const orc_mesh *m, int64_t c, int i)
{
    return m->nodes + (int64_t)m->cells[c * (m->dim + 1) + i] * m->dim;
}

/* Barycentric coordinates by their definition as ratios of signed measures:
 * lambda_i = measure(cell with vertex i replaced by x) / measure(cell). */
static void barycentric(const orc_mesh *m, int64_t c, const double *x, double *lam)
{
    const double *v0 = mesh_node(m, c, 0), *v1 = mesh_node(m, c, 1), *v2 = mesh_node(m, c, 2);
    if (m->dim == 2) {
        double A = area2(v0, v1, v2);
        lam[0] = area2(x, v1, v2) / A;
        lam[1] = area2(v0, x, v2) / A;
        lam[2] = area2(v0, v1, x) / A;
        lam[3] = 0.0;
    } else {
        const double *v3 = mesh_node(m, c, 3);
        double V = vol6(v0, v1, v2, v3);
        lam[0] = vol6(x, v1, v2, v3) / V;
        lam[1] = vol6(v0, x, v2, v3) / V;
        lam[2] = vol6(v0, v1, x, v3) / V;
        lam[3] = vol6(v0, v1, v2, x) / V;
    }
}

static int64_t bucket_axis(const orc_mesh *m, int a, double x)
{
    double q = floor((x - m->lo[a]) / m->bsize[a]);
    if (q < 0.0) return 0;
    if (q > (double)(m->nb[a] - 1)) return m->nb[a] - 1;
    return (int64_t)q;
}

static int64_t bucket_id(const orc_mesh *m, const int64_t *b)
{
    return b[0] + m->nb[0] * (b[1] + m->nb[1] * b[2]);
}

orc_mesh *orc_mesh_new(int32_t dim, int64_t n_nodes, const double *nodes, int64_t n_cells,
                       const int32_t *cells, int32_t n_frames, double t_first, double dt_frame,
                       const double *u)
{
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    if (!m) return NULL;
    m->dim = dim;
    m->n_frames = n_frames;
    m->n_nodes = n_nodes;
    m->n_cells = n_cells;
    m->nodes = nodes;
    m->cells = cells;
    m->t_first = t_first;
    m->dt_frame = dt_frame;
    m->u = u;
    m->tol = 1e-12;
    for (int a = 0; a < 3; ++a) {
        m->lo[a] = 0.0;
        m->hi[a] = 0.0;
        m->nb[a] = 1;
        m->bsize[a] = 1.0;
    }
    for (int a = 0; a < dim; ++a) {
        m->lo[a] = INFINITY;
        m->hi[a] = -INFINITY;
    }
    for (int64_t p = 0; p < n_nodes; ++p)
        for (int a = 0; a < dim; ++a) {
            double x = nodes[p * dim + a];
            if (x < m->lo[a]) m->lo[a] = x;
            if (x > m->hi[a]) m->hi[a] = x;
        }
    /* buckets of about two cells each */
    double vol = 1.0;
    for (int a = 0; a < dim; ++a) vol *= (m->hi[a] - m->lo[a]);
    double edge = pow(2.0 * vol / (double)n_cells, 1.0 / (double)dim);
    for (int a = 0; a < dim; ++a) {
        double ext = m->hi[a] - m->lo[a];
        int64_t k = (int64_t)ceil(ext / edge);
        m->nb[a] = k < 1 ? 1 : k;
        m->bsize[a] = ext / (double)m->nb[a];
    }
    int64_t nbt = m->nb[0] * m->nb[1] * m->nb[2];
    m->bstart = (int64_t *)calloc((size_t)nbt + 1, sizeof(int64_t));
    int64_t (*range)[2][3] = malloc((size_t)n_cells * sizeof(*range));
    if (!m->bstart || !range) {
        free(range);
        free(m->bstart);
        free(m);
        return NULL;
    }
    for (int64_t c = 0; c < n_cells; ++c) {
        for (int a = 0; a < 3; ++a) {
            range[c][0][a] = 0;
            range[c][1][a] = 0;
        }
        for (int a = 0; a < dim; ++a) {
            double cmin = INFINITY, cmax = -INFINITY;
            for (int i = 0; i <= dim; ++i) {
                double x = mesh_node(m, c, i)[a];
                if (x < cmin) cmin = x;
                if (x > cmax) cmax = x;
            }
            double slack = 1e-9 * (m->hi[a] - m->lo[a]);
            range[c][0][a] = bucket_axis(m, a, cmin - slack);
            range[c][1][a] = bucket_axis(m, a, cmax + slack);
        }
        int64_t b[3];
        for (b[2] = range[c][0][2]; b[2] <= range[c][1][2]; ++b[2])
            for (b[1] = range[c][0][1]; b[1] <= range[c][1][1]; ++b[1])
                for (b[0] = range[c][0][0]; b[0] <= range[c][1][0]; ++b[0])
                    m->bstart[bucket_id(m, b) + 1] += 1;
    }
    for (int64_t q = 0; q < nbt; ++q) m->bstart[q + 1] += m->bstart[q];
    m->bcells = (int32_t *)malloc((size_t)(m->bstart[nbt] > 0 ? m->bstart[nbt] : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)calloc((size_t)nbt, sizeof(int64_t));
    if (!m->bcells || !fill) {
        free(fill);
        free(range);
        free(m->bcells);
        free(m->bstart);
        free(m);
        return NULL;
    }
    for (int64_t c = 0; c < n_cells; ++c) {     /* ascending cell ids in every bucket */
        int64_t b[3];
        for (b[2] = range[c][0][2]; b[2] <= range[c][1][2]; ++b[2])
            for (b[1] = range[c][0][1]; b[1] <= range[c][1][1]; ++b[1])
                for (b[0] = range[c][0][0]; b[0] <= range[c][1][0]; ++b[0]) {
                    int64_t q = bucket_id(m, b);
                    m->bcells[m->bstart[q] + fill[q]++] = (int32_t)c;
                }
    }
    free(fill);
    free(range);
    return m;
}

void orc_mesh_free(orc_mesh *m)
{
    if (!m) return;
    free(m->bcells);
    free(m->bstart);
    free(m);
}

/* The cell holding x: among the cells listed in x's bucket, the one whose
 * smallest barycentric coordinate is largest (the most interior one; equal
 * values go to the lower cell id), accepted if that coordinate is >= -tol.
 * Returns the cell id and its barycentric coordinates, or -1 outside. */
int64_t orc_mesh_locate(const orc_mesh *m, const double *x, double *lam_out)
{
    for (int a = 0; a < m->dim; ++a) {
        if (!isfinite(x[a])) return -1;
        double slack = 1e-9 * (m->hi[a] - m->lo[a]);
        if (x[a] < m->lo[a] - slack || x[a] > m->hi[a] + slack) return -1;
    }
    int64_t b[3] = {0, 0, 0};
    for (int a = 0; a < m->dim; ++a) b[a] = bucket_axis(m, a, x[a]);
    int64_t q = bucket_id(m, b);
    int64_t best = -1;
    double best_min = -INFINITY, best_lam[4] = {0, 0, 0, 0};
    for (int64_t s = m->bstart[q]; s < m->bstart[q + 1]; ++s) {
        int64_t c = m->bcells[s];
        double lam[4];
        barycentric(m, c, x, lam);
        double mn = lam[0];
        for (int i = 1; i <= m->dim; ++i)
            if (lam[i] < mn) mn = lam[i];
        if (best < 0 || mn > best_min) {
            best = c;
            best_min = mn;
            for (int i = 0; i < 4; ++i) best_lam[i] = lam[i];
        }
    }
    if (best < 0 || !(best_min >= -m->tol)) return -1;
    if (lam_out)
        for (int i = 0; i < 4; ++i) lam_out[i] = best_lam[i];
    return best;
}

void orc_mesh_locate_many(const orc_mesh *m, const double *x, int64_t n, int64_t *cell,
                          double *lam)
{
    for (int64_t p = 0; p < n; ++p) {
        double q[3] = {0, 0, 0}, l[4] = {0, 0, 0, 0};
        for (int a = 0; a < m->dim; ++a) q[a] = x[a * n + p];
        int64_t c = orc_mesh_locate(m, q, l);
        cell[p] = c;
        if (lam)
            for (int i = 0; i <= m->dim; ++i) lam[i * n + p] = c >= 0 ? l[i] : NAN;
    }
}

/* Frame pair bracketing t (same rule as on structured grids). */
static void mesh_frame_pair(const orc_mesh *m, double t, int64_t *f, double *alpha)
{
    double q = floor((t - m->t_first) / m->dt_frame);
    int64_t fi = (int64_t)q;
    if (fi > m->n_frames - 2) fi = m->n_frames - 2;
    if (fi < 0) fi = 0;
    double tf = m->t_first + (double)fi * m->dt_frame;
    *f = fi;
    *alpha = (t - tf) / m->dt_frame;
}

/* u(x, t) = (1 - alpha) sum_i lambda_i u_f(node_i) + alpha sum_i lambda_i
 * u_{f+1}(node_i).  Returns 0 (and leaves out untouched) if x is in no cell. */
int orc_mesh_velocity_at(const orc_mesh *m, const double *x, double t, double *out)
{
    double lam[4];
    int64_t c = orc_mesh_locate(m, x, lam);
    if (c < 0) return 0;
    int64_t f;
    double alpha;
    mesh_frame_pair(m, t, &f, &alpha);
    int d = m->dim;
    for (int k = 0; k < d; ++k) {
        double s0 = 0.0, s1 = 0.0;
        for (int i = 0; i <= d; ++i) {
            int64_t node = m->cells[c * (d + 1) + i];
            s0 += lam[i] * m->u[(f * m->n_nodes + node) * d + k];
            s1 += lam[i] * m->u[((f + 1) * m->n_nodes + node) * d + k];
        }
        out[k] = (1.0 - alpha) * s0 + alpha * s1;
    }
    return 1;
}

void orc_mesh_velocity_at_many(const orc_mesh *m, const double *x, const double *t, int64_t n,
                               double *out, uint8_t *found)
{
    for (int64_t p = 0; p < n; ++p) {
        double q[3] = {0, 0, 0}, r[3] = {NAN, NAN, NAN};
        for (int a = 0; a < m->dim; ++a) q[a] = x[a * n + p];
        int ok = orc_mesh_velocity_at(m, q, t[p], r);
        if (found) found[p] = (uint8_t)ok;
        for (int a = 0; a < m->dim; ++a) out[a * n + p] = r[a];
    }
}

/* Check a stage point or a new position: non-finite -> NONFINITE, in no cell
 * of the mesh -> OUT.  margin (diagnostic): the smallest distance, inside or
 * outside, of a checked point to a face of the mesh's bounding box, which is
 * its distance to the boundary for the box-shaped meshes this oracle is used
 * with. */
static uint32_t mesh_check_point(const orc_mesh *m, const double *p, double *margin)
{
    if (!all_finite(p, m->dim)) return ORC_FLAG_NONFINITE;
    if (margin)
        for (int a = 0; a < m->dim; ++a) {
            double d = fmin(fabs(p[a] - m->lo[a]), fabs(m->hi[a] - p[a]));
            if (d < *margin) *margin = d;
        }
    if (orc_mesh_locate(m, p, NULL) < 0) return ORC_FLAG_OUT;
    return 0;
}

/* Classical RK4 step on the mesh field; the same exit reading as on
 * structured grids (a rejected step leaves x unchanged). */
static uint32_t mesh_rk4_step(const orc_mesh *m, double *x, double t, double dt, double *margin)
{
    int d = m->dim;
    double k1[3], k2[3], k3[3], k4[3], p[3], xn[3];
    uint32_t fl;

    if (!orc_mesh_velocity_at(m, x, t, k1)) return ORC_FLAG_OUT;
    if (!all_finite(k1, d)) return ORC_FLAG_NONFINITE;

    for (int a = 0; a < d; ++a) p[a] = x[a] + 0.5 * dt * k1[a];
    if ((fl = mesh_check_point(m, p, margin))) return fl;
    orc_mesh_velocity_at(m, p, t + 0.5 * dt, k2);
    if (!all_finite(k2, d)) return ORC_FLAG_NONFINITE;

    for (int a = 0; a < d; ++a) p[a] = x[a] + 0.5 * dt * k2[a];
    if ((fl = mesh_check_point(m, p, margin))) return fl;
    orc_mesh_velocity_at(m, p, t + 0.5 * dt, k3);
    if (!all_finite(k3, d)) return ORC_FLAG_NONFINITE;

    for (int a = 0; a < d; ++a) p[a] = x[a] + dt * k3[a];
    if ((fl = mesh_check_point(m, p, margin))) return fl;
    orc_mesh_velocity_at(m, p, t + dt, k4);
    if (!all_finite(k4, d)) return ORC_FLAG_NONFINITE;

    for (int a = 0; a < d; ++a)
        xn[a] = x[a] + (dt / 6.0) * (k1[a] + 2.0 * k2[a] + 2.0 * k3[a] + k4[a]);
    if ((fl = mesh_check_point(m, xn, margin))) return fl;

    for (int a = 0; a < d; ++a) x[a] = xn[a];
    return 0;
}

static int mesh_time_span_ok(const orc_mesh *m, double t0, double T)
{
    double t_last = m->t_first + (double)(m->n_frames - 1) * m->dt_frame;
    double t1 = t0 + T;
    return t0 >= m->t_first && t0 <= t_last && t1 >= m->t_first && t1 <= t_last;
}

/* One tracer from x (in place): flags as on structured grids.  lam_margin
 * (diagnostic): the smallest barycentric coordinate of the final position in
 * its cell (how close it sits to a face), -inf if it is in no cell. */
static uint32_t mesh_advect_one(const orc_mesh *m, double *x, double t0, double T, double dt,
                                double *margin, int64_t *cell, double *lam_margin)
{
    uint32_t fl = mesh_time_span_ok(m, t0, T) ? mesh_check_point(m, x, margin) : ORC_FLAG_TIME_OUT;
    int64_t nsteps = step_count(T, dt);
    for (int64_t n = 0; n < nsteps && !fl; ++n)
        fl = mesh_rk4_step(m, x, t0 + (double)n * dt, dt, margin);
    double lam[4];
    *cell = orc_mesh_locate(m, x, lam);
    double mn = -INFINITY;
    if (*cell >= 0) {
        mn = lam[0];
        for (int i = 1; i <= m->dim; ++i)
            if (lam[i] < mn) mn = lam[i];
    }
    *lam_margin = mn;
    return fl;
}

/* Advect the seeds of a (non-periodic) structured seed grid, or the listed
 * ones (idx != NULL), from t0 over T with step dt.  Outputs as for
 * orc_advect_seeds; cell = the mesh cell holding the final position (-1 if
 * none).  Any output may be NULL. */
void orc_mesh_advect_seeds(const orc_mesh *m, const orc_seed_grid *g, const int64_t *idx,
                           int64_t n, double t0, double T, double dt, double *xf, int64_t *cell,
                           uint8_t *flags, double *margin, double *lam_margin, int nthreads)
{
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t p = 0; p < n; ++p) {
        double x[3] = {0, 0, 0};
        seed_position(g, idx ? idx[p] : p, x);
        double mg = INFINITY, lm;
        int64_t c;
        uint32_t fl = mesh_advect_one(m, x, t0, T, dt, &mg, &c, &lm);
        if (xf)
            for (int a = 0; a < m->dim; ++a) xf[a * n + p] = x[a];
        if (cell) cell[p] = c;
        if (flags) flags[p] = (uint8_t)fl;
        if (margin) margin[p] = mg;
        if (lam_margin) lam_margin[p] = lm;
    }
    (void)nthreads;
}

/* Advect arbitrary points x0 (dim x n), each from its own t0[p]. */
void orc_mesh_advect_points(const orc_mesh *m, const double *x0, const double *t0, int64_t n,
                            double T, double dt, double *xf, int64_t *cell, uint8_t *flags,
                            double *margin, double *lam_margin, int nthreads)
{
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
    for (int64_t p = 0; p < n; ++p) {
        double x[3] = {0, 0, 0};
        for (int a = 0; a < m->dim; ++a) x[a] = x0[a * n + p];
        double mg = INFINITY, lm;
        int64_t c;
        uint32_t fl = mesh_advect_one(m, x, t0[p], T, dt, &mg, &c, &lm);
        if (xf)
            for (int a = 0; a < m->dim; ++a) xf[a * n + p] = x[a];
        if (cell) cell[p] = c;
        if (flags) flags[p] = (uint8_t)fl;
        if (margin) margin[p] = mg;
        if (lam_margin) lam_margin[p] = lm;
    }
    (void)nthreads;
}
