/*
 * lcs.h -- C ABI of the MI355X (gfx950) LCS flow-map / FTLE library.
 *
 * Method: Ameli, Desai & Shadden, "Development of an efficient and flexible
 * pipeline for Lagrangian coherent structure computation".  The library
 * implements the data-parallel hot path of that pipeline:
 *
 *   seed grid (Sec. 2, Seed filter)
 *     -> RK4 advection through gridded, time-dependent velocity frames with
 *        space-time interpolation (Eq. 2; Sec. 2 Interpolator and Flow Map
 *        filters; Sec. 3.1)
 *     -> flow-map gradient by central differences on the seed grid and the
 *        Cauchy-Green tensor C = grad(F)^T grad(F) (Eq. 1; Sec. 2 Cauchy-Green
 *        filter)
 *     -> largest eigenvalue of C and the FTLE (Sec. 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers marked [device] are HIP device pointers (HBM); [host] are host
 *   pointers.  The caller owns every buffer; the library keeps no pointer after
 *   a call returns, except where a plan says otherwise.
 * - Arrays are contiguous and dense.  Outputs must not alias inputs.
 * - Vector fields over N points are structure-of-arrays: component a of point
 *   p is at [a*N + p].  Seed-grid arrays are in natural seed order (x index
 *   fastest, then y, then z).
 * - Every call validates all arguments on the host BEFORE anything is
 *   launched; a non-OK status means nothing was enqueued or written.
 * - Work is enqueued asynchronously on the caller's stream (hipStream_t passed
 *   as void*, NULL = the default stream).  A kernel fault surfaces as
 *   LCS_E_HIP from a later call or from lcs_sync_status().
 * - lcs_last_error() returns a thread-local description of the last non-OK
 *   status returned on the calling thread.
 * - Advection arithmetic is FP32; the gradient, C, lambda_max and the FTLE are
 *   FP64.
 */
#ifndef LCS_H
#define LCS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LCS_OK = 0,
    LCS_E_ARG = -1,          /* NULL required pointer, bad dim, bad count          */
    LCS_E_SHAPE = -2,        /* grid sizes out of the supported range              */
    LCS_E_TIME_RANGE = -3,   /* [t0, t0+T] leaves the span of the frames           */
    LCS_E_SEED_DOMAIN = -4,  /* a seed lies outside a non-periodic velocity axis   */
    LCS_E_STEP = -5,         /* T/dt not integral, sign(dt) != sign(T), or T == 0  */
    LCS_E_HIP = -6,          /* HIP launch or runtime failure                      */
    LCS_E_UNSUPPORTED = -7   /* valid request the library does not handle         */
} lcs_status;

/* Per-tracer flag bits (uint8). */
enum {
    LCS_FLAG_OUT = 1u,         /* a stage point or new position left the closed domain */
    LCS_FLAG_NONFINITE = 2u,   /* a position or sampled velocity was not finite         */
    LCS_FLAG_STENCIL_OUT = 4u, /* (C / FTLE) a tracer of the difference stencil is flagged */
    LCS_FLAG_TIME_OUT = 8u,    /* (points) the tracer's interval leaves the frame span  */
    LCS_FLAG_LOST = 16u        /* (meshes) the local cell search hit its step limit     */
};

/*
 * Gridded, time-dependent velocity data (Sec. 2 Interpolator filter: the
 * frames are held in GPU memory; here every frame stays resident in HBM).
 *
 * dim          2 or 3.
 * n[a]         nodes along axis a (n[2] == 1 in 2D); n[a] >= 2, and
 *              n0*n1*n2 < 2^31; one frame of one array (a component in
 *              LCS_LAYOUT_SOA, all components when interleaved) must be at
 *              most 4 GiB (n0*n1*n2 * 4 B, resp. * 4*dim B or * 16 B), else
 *              LCS_E_SHAPE.
 * origin[a],   node i of axis a sits at origin[a] + i*spacing[a].
 * spacing[a]   spacing[a] > 0.
 * periodic_mask  bit a set: axis a is periodic with period n[a]*spacing[a]
 *              (no duplicated end node).  Otherwise the domain along a is the
 *              closed interval [origin, origin + (n-1)*spacing].
 * n_frames     >= 2; frame f holds the field at t_first + f*dt_frame,
 *              dt_frame > 0.
 * layout       how the frames are stored (node = i + n0*(j + n1*k),
 *              N = n0*n1*n2):
 *   LCS_LAYOUT_SOA   u[c] [device] FP32, component c of all frames at
 *                    u[c][f*N + node] (structure of arrays); u[2] ignored in 2D.
 *   LCS_LAYOUT_XYZ   u[0] [device] FP32, the dim components of a node adjacent:
 *                    u[0][(f*N + node)*dim + c] (interleaved, as VTK stores
 *                    vector point data); u[1], u[2] ignored; 4-byte aligned
 *                    (8-byte in 2D).
 *   LCS_LAYOUT_XYZW  3D only: u[0][(f*N + node)*4 + c], the 4th float unused;
 *                    16-byte aligned.
 *   LCS_LAYOUT_TPAIR time-paired records: for each frame pair (p, p+1),
 *                    p < n_frames-1, and each node of a grid with one extra
 *                    x node (n0+1 per row; the extra node repeats node 0 of
 *                    the row), the dim floats of frame p then those of frame
 *                    p+1:  u[0][(((p*n2 + k)*n1 + j)*(n0+1) + i)*2*dim + c'],
 *                    c' < dim frame p, c' >= dim frame p+1; 16-byte aligned;
 *                    (n_frames-1)*(n0+1)*n1*n2*8*dim bytes.  The two x nodes
 *                    of a cell row and both frames are then 16*dim contiguous
 *                    bytes.
 *              Every layout gives the same field; the interleaved ones need
 *              fewer memory transactions per interpolation (one record per
 *              node instead of one value per component array), see
 *              lcs_frames_interleave.
 */
enum {
    LCS_LAYOUT_SOA = 0,
    LCS_LAYOUT_XYZ = 1,
    LCS_LAYOUT_XYZW = 2,
    LCS_LAYOUT_TPAIR = 3
};

typedef struct {
    int32_t dim;
    int32_t n_frames;
    int64_t n[3];
    double origin[3];
    double spacing[3];
    uint32_t periodic_mask;
    uint32_t layout;          /* LCS_LAYOUT_* */
    double t_first;
    double dt_frame;
    const float *u[3];
} lcs_velocity_t;

/*
 * Structured seed grid (Sec. 2 Seed filter): seed (i,j,k) starts at
 * origin + (i,j,k)*spacing.  A periodic seed axis (bit a of periodic_mask)
 * has period n[a]*spacing[a], which must equal the velocity period on that
 * axis; the gradient then differences across the seam.  n[a] >= 2 on every
 * axis < dim, n[2] == 1 in 2D.
 */
typedef struct {
    int32_t dim;
    uint32_t periodic_mask;
    int64_t n[3];
    double origin[3];
    double spacing[3];
} lcs_seed_grid_t;

/* One integration window of a batched call: start time and signed duration. */
typedef struct {
    double t0;
    double T;
} lcs_window_t;

/* Opaque plan: device state the library owns for batched launches (a work
 * counter, a capture stream and the captured HIP graph) and the autotuner's
 * choices (lcs_advect_tuned).  One plan per device and per host thread at a
 * time; calls that share a plan must not overlap. */
typedef struct lcs_plan *lcs_plan_t;

/* Maximum number of windows of one lcs_advect_batched call. */
#define LCS_MAX_WINDOWS 192

/* Maximum number of snapshots of one lcs_advect_snapshots call. */
#define LCS_MAX_SNAPSHOTS 64

/*
 * lcs_frames_interleave -- copy frames f_first .. f_first+f_count-1 of a
 * structure-of-arrays velocity (layout LCS_LAYOUT_SOA) into an interleaved
 * layout (LCS_LAYOUT_XYZ or LCS_LAYOUT_TPAIR; in 3D also LCS_LAYOUT_XYZW) on
 * the device, and describe the copy (Sec. 2 Reader/Cache filters: velocity
 * data staged in GPU memory in the form the kernels read).
 * out       [device] FP32, lcs_frames_interleave_floats(soa, layout, f_count)
 *           floats, aligned as the layout requires.
 * out_desc  [host] filled with the interleaved descriptor of the copied span
 *           (t_first moved to frame f_first, n_frames = f_count >= 2).
 */
lcs_status lcs_frames_interleave(const lcs_velocity_t *soa, uint32_t layout, int32_t f_first,
                                 int32_t f_count, float *out, lcs_velocity_t *out_desc,
                                 void *stream);

/* Floats that f_count frames of soa's grid occupy in an interleaved layout
 * (f_count * N * S for XYZ / XYZW; (f_count-1) * (n0+1)*n1*n2 * 2*dim for TPAIR),
 * or -1 for an invalid layout, dimension or f_count < 2. */
int64_t lcs_frames_interleave_floats(const lcs_velocity_t *soa, uint32_t layout, int32_t f_count);

/*
 * lcs_advect -- flow map F_{t0}^{t0+T} of a structured seed grid (Eq. 2;
 * Sec. 2 Seed and Flow Map filters; Sec. 3.1 RK4).
 *
 * Every seed is integrated with N = T/dt classical RK4 steps,
 * t_n = t0 + n*dt, through the velocity interpolated multilinearly in space
 * and linearly in time between the two frames bracketing t.  Backward
 * integration uses T < 0, dt < 0.  Positions on periodic axes are unwrapped.
 * A tracer whose stage point or new position leaves the closed domain (or
 * meets a non-finite value) is frozen at its last accepted position and
 * flagged.  Seeds are generated on the device from the descriptor.
 *
 * xf     [device] FP32, dim x Ns (Ns = n0*n1*n2), final positions.
 * cell   [device] int64, Ns, or NULL: lower-corner linear index
 *        i + n0*(j + n1*k) of the velocity cell holding the final position,
 *        computed in FP64 from the returned FP32 position.
 * flags  [device] uint8, Ns, or NULL: LCS_FLAG_OUT / LCS_FLAG_NONFINITE.
 * Errors: LCS_E_ARG, LCS_E_SHAPE, LCS_E_TIME_RANGE, LCS_E_SEED_DOMAIN,
 *         LCS_E_STEP, LCS_E_HIP.
 */
lcs_status lcs_advect(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds,
                      double t0, double T, double dt,
                      float *xf, int64_t *cell, uint8_t *flags, void *stream);

/*
 * lcs_advect_sorted -- lcs_advect with re-bundled tracers: the integration
 * runs in segments of `segment_steps` RK4 steps (0 = 50); before the first and
 * between segments the tracers are counting-sorted by the Morton code of the
 * 2 x 2 (x 2) velocity-cell bin they occupy, so that the lanes of a wavefront
 * gather from one compact region although trajectories spread apart.  The
 * per-tracer arithmetic is that of lcs_advect, so xf / cell / flags are
 * bit-identical to it.  (The paper observed that tracers with neighbouring
 * memory indices stop being neighbours in space, Sec. 3.2, and cites
 * spatially coherent re-bundling as a remedy.)
 *
 * workspace [device] of at least lcs_advect_sorted_workspace_bytes(vel, seeds)
 * bytes (about 70 B per seed plus 4 B per sort bin): two copies of the tracer
 * state, each slot's key and rank within its key, the permutation, the bin
 * histogram.  Other arguments and errors as lcs_advect.
 */
int64_t lcs_advect_sorted_workspace_bytes(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds);
lcs_status lcs_advect_sorted(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds,
                             double t0, double T, double dt, int32_t segment_steps,
                             float *xf, int64_t *cell, uint8_t *flags,
                             void *workspace, int64_t workspace_bytes, void *stream);

/*
 * lcs_advect_sorted_noalloc -- lcs_advect_sorted for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the re-bundling workspace is a fixed
 * device array inside the library, LCS_NOALLOC_SCRATCH_BYTES (64 MiB) per
 * device, held from library load until the process ends.  No hipMalloc,
 * hipFree or other allocation happens in the call.  Same arithmetic and
 * results as lcs_advect_sorted (bit-identical to lcs_advect).
 * Every call on one device uses the same array and leaves its contents there
 * (the histogram is cleared at the start of each call): calls that overlap on
 * one device -- on different streams or host threads -- race and give wrong
 * results; serialise them.
 * Errors: those of lcs_advect_sorted, and LCS_E_SHAPE when the grid needs
 * more workspace than the array holds (lcs_advect_sorted_workspace_bytes >
 * LCS_NOALLOC_SCRATCH_BYTES; about 70 B per seed plus 4 B per sort bin).
 */
#define LCS_NOALLOC_SCRATCH_BYTES (64LL << 20)
lcs_status lcs_advect_sorted_noalloc(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds,
                                     double t0, double T, double dt, int32_t segment_steps,
                                     float *xf, int64_t *cell, uint8_t *flags, void *stream);

/*
 * lcs_advect_points -- flow map of arbitrary points, each with its own start
 * time (Eq. 2): the same integrator as lcs_advect over the duration T.
 * Used to resume segments, to draw check samples and to produce training
 * pairs for the surrogate.
 *
 * x0     [device] FP32, dim x n, start positions.
 * t0     [device] FP64, n, start time of each point.  A point whose
 *        interval [t0, t0+T] leaves the frame span is not advected and gets
 *        LCS_FLAG_TIME_OUT (its xf is x0).
 * xf, cell, flags as in lcs_advect (cell and flags may be NULL).
 * n must be in [1, 2^31-1] (LCS_E_SHAPE otherwise, as for lcs_ftle).
 * Errors: LCS_E_ARG, LCS_E_SHAPE, LCS_E_STEP, LCS_E_HIP.
 */
lcs_status lcs_advect_points(const lcs_velocity_t *vel, const float *x0, const double *t0,
                             int64_t n, double T, double dt,
                             float *xf, int64_t *cell, uint8_t *flags, void *stream);

/*
 * lcs_cg_tensor -- Cauchy-Green tensor on the seed grid (Eq. 1; Sec. 2
 * Cauchy-Green filter: central differences of the final positions over the
 * seed grid).
 *
 * grad F is formed in FP64 from the FP32 positions: central differences
 * (F(x+h e_b) - F(x-h e_b)) / (2h) in the interior and on periodic axes (the
 * neighbour across a seam is shifted by the period along its own axis),
 * first-order one-sided differences on the first and last seed of a
 * non-periodic axis.  C = grad(F)^T grad(F).
 *
 * xf            [device] FP32, dim x Ns, as written by lcs_advect.
 * flags         [device] uint8, Ns, or NULL: tracer flags from lcs_advect.
 * C             [device] FP64, packed symmetric, nq x Ns with nq = 3 (2D:
 *               xx, xy, yy) or 6 (3D: xx, xy, xz, yy, yz, zz).
 * stencil_flags [device] uint8, Ns, or NULL: LCS_FLAG_STENCIL_OUT where the
 *               seed or a neighbour it differences carries a flag.
 * Errors: LCS_E_ARG, LCS_E_SHAPE, LCS_E_HIP.
 */
lcs_status lcs_cg_tensor(const lcs_seed_grid_t *seeds, const float *xf, const uint8_t *flags,
                         double *C, uint8_t *stencil_flags, void *stream);

/*
 * lcs_ftle -- largest eigenvalue of C and the FTLE field (Sec. 1: the FTLE
 * derives from the largest eigenvalue of C; Sec. 2 Cauchy-Green filter).
 *
 * sigma = ln(lambda_max) / (2|T|); lambda_max <= 0 gives -inf.  FP64.
 * dim         2 or 3.   n_points >= 1.
 * C           [device] FP64 packed, nq x n_points (layout of lcs_cg_tensor).
 * lambda_max  [device] FP64, n_points, or NULL.
 * ftle        [device] FP64, n_points, or NULL (not both NULL).
 * Errors: LCS_E_ARG, LCS_E_HIP.
 */
lcs_status lcs_ftle(int32_t dim, int64_t n_points, const double *C, double T,
                    double *lambda_max, double *ftle, void *stream);

/*
 * lcs_cg_ftle -- lcs_cg_tensor followed by lcs_ftle in one pass, without
 * materialising C (same arithmetic, same results).  For large seed grids.
 * lambda_max, ftle, stencil_flags [device] FP64/FP64/uint8, Ns, each may be
 * NULL but not lambda_max and ftle both.
 * Errors: LCS_E_ARG, LCS_E_SHAPE, LCS_E_HIP.
 */
lcs_status lcs_cg_ftle(const lcs_seed_grid_t *seeds, const float *xf, const uint8_t *flags,
                       double T, double *lambda_max, double *ftle, uint8_t *stencil_flags,
                       void *stream);

/*
 * lcs_advect_batched -- the flow map of one seed grid for a time series of
 * start times (Sec. 1: the FTLE field of a flow is usually wanted for many
 * start times; Sec. 4: sampling is dense in space, not in time), all windows
 * in ONE persistent launch replayed from a HIP graph.
 *
 * Window w integrates N_w = T_w/dt RK4 steps from windows[w].t0 (same
 * integrator, same outputs as lcs_advect, bit-identical to calling lcs_advect
 * per window).  Work items are (window, seed tile) pairs, windows in order of
 * start time; the tiles are split into 8 contiguous runs along the Morton
 * curve, one per XCD, each drained from its own device counter by that XCD's
 * persistent workgroups (each XCD then reads one compact part of the domain).
 * The (counter reset,
 * kernel) pair is captured once into a graph on a plan-owned stream and
 * replayed on `stream`; a call whose arguments differ from the captured ones
 * re-captures.
 *
 * plan      from lcs_plan_create (must be the current device's).
 * windows   [host] n_windows entries, 1 <= n_windows <= LCS_MAX_WINDOWS; every
 *           window inside the frame span; sign(T_w) == sign(dt); T_w/dt integral.
 * xf        [device] FP32, n_windows x dim x Ns (window-major, caller's order).
 * cell      [device] int64, n_windows x Ns, or NULL.
 * flags     [device] uint8, n_windows x Ns, or NULL.
 * Errors: LCS_E_ARG, LCS_E_SHAPE, LCS_E_TIME_RANGE, LCS_E_SEED_DOMAIN,
 *         LCS_E_STEP, LCS_E_HIP.
 */
lcs_status lcs_advect_batched(lcs_plan_t plan, const lcs_velocity_t *vel,
                              const lcs_seed_grid_t *seeds, const lcs_window_t *windows,
                              int32_t n_windows, double dt, float *xf, int64_t *cell,
                              uint8_t *flags, void *stream);

/* lcs_plan_create / lcs_plan_destroy -- allocate / free a plan on the current
 * device (hipMalloc of 8 four-byte work counters, one non-blocking stream).
 * autotune_cache_path [host] NUL-terminated file name or NULL: the
 * autotuner's choices are read from it now (one JSON object per line, as
 * lcs_advect_tuned appends them; a missing file is an empty cache) and every
 * new choice is appended to it.  lcs_plan_destroy waits for the plan's stream
 * and accepts NULL. */
lcs_status lcs_plan_create(lcs_plan_t *plan, const char *autotune_cache_path);
lcs_status lcs_plan_destroy(lcs_plan_t plan);

/* lcs_plan_stats -- number of graph launches and graph captures so far
 * (either pointer may be NULL). */
lcs_status lcs_plan_stats(lcs_plan_t plan, int64_t *graph_launches, int64_t *graph_captures);

/*
 * lcs_advect_tuned -- lcs_advect with the seed ordering picked by the plan's
 * autotuner (the tracer locality the paper found decisive, Sec. 3.2, depends
 * on the field and the seed grid, so the choice is measured, not fixed).
 * Candidates are segment lengths: 0 = the single launch of lcs_advect,
 * S > 0 = lcs_advect_sorted re-bundling every S steps; NULL takes
 * {0, 200, 100, 50, 25}.  The first call for a workload key (device
 * architecture, velocity grid, layout, periodicity and frame count, seed grid,
 * step count and direction) runs the first runnable candidate once untimed,
 * then every runnable candidate once, timed with HIP events on `stream`
 * (this call synchronises), keeps the fastest in the plan and appends it to
 * the plan's cache file; later calls for that key (also in a later process
 * through the cache) run the choice directly, asynchronously.  Re-bundled
 * candidates need `workspace` of lcs_advect_sorted_workspace_bytes (else they
 * are skipped, and a cached re-bundled choice falls back to the single
 * launch).  Every candidate computes the same bits, so xf / cell / flags are
 * those of lcs_advect whatever the choice.
 * chosen        [host] int32 or NULL: the segment length that ran (0 = single).
 * candidate_ms  [host] FP32 x n_candidates or NULL: on a tuning call, each
 *               candidate's time (NaN if skipped); untouched otherwise.
 * Errors: LCS_E_ARG (NULL plan, plan of another device, n_candidates outside
 *   1..16, a negative candidate, no runnable candidate) and those of
 *   lcs_advect / lcs_advect_sorted.
 */
lcs_status lcs_advect_tuned(lcs_plan_t plan, const lcs_velocity_t *vel,
                            const lcs_seed_grid_t *seeds, double t0, double T, double dt,
                            float *xf, int64_t *cell, uint8_t *flags, void *workspace,
                            int64_t workspace_bytes, const int32_t *candidates,
                            int32_t n_candidates, int32_t *chosen, float *candidate_ms,
                            void *stream);

/* ------------------------------------------------------------------------
 * Learned flow-map surrogate: a Fourier-feature MLP that predicts the
 * displacement of a point over a window tau (a local approximation of the
 * flow map; the paper's discussion cites such approximations as a way to cut
 * interpolation work when flow maps are wanted for many start times, Sec. 4).
 * Plain RK4 remains the reference and the fallback.
 *
 * Fixed architecture: input (x, y, z, t) -> v = (input - in_shift) * in_scale
 * -> 128 features [cos(2 pi B v), sin(2 pi B v)] (B: 64 x 4) -> 4 hidden
 * layers of 256 with the tanh form of GELU -> 3 outputs -> displacement =
 * out_scale * output.  Hidden-layer products run on BF16 MFMA with FP32
 * accumulation; features, biases, head and loss are FP32.
 *
 * FP32 master parameters, one flat vector of LCS_MLP_PARAMS values:
 *   W_0 [128][256] (row-major [in][out]), b_0 [256],
 *   W_l [256][256], b_l [256] for l = 1, 2, 3,
 *   W_h [256][3], b_h [3].
 * BF16 compute copies (LCS_MLP_BF16 values, written by lcs_mlp_refresh_bf16):
 *   for l = 0..3: W_l ([in][out]: R = in rows of C = 256 values), then W_l^T
 *   ([out][in]: R = 256 rows of C = in values), each in MFMA fragment order:
 *   element (r, c) at ((r/16)*(C/32) + c/32)*512 + ((r%16) + 16*((c%32)/8))*8
 *   + c%8, so that each 16 x 32 block is 64 lanes x 8 consecutive c, one
 *   contiguous 1 KiB.
 * ------------------------------------------------------------------------ */
#define LCS_MLP_FREQ 64
#define LCS_MLP_WIDTH 256
#define LCS_MLP_HIDDEN 4
#define LCS_MLP_PARAMS 231171
#define LCS_MLP_BF16 458752

typedef struct {
    const float *freq;              /* [device] FP32, LCS_MLP_FREQ x 4, row-major */
    float in_shift[4];
    float in_scale[4];
    float out_scale;
    uint32_t reserved;              /* must be 0 */
    const float *params;            /* [device] FP32 masters, LCS_MLP_PARAMS */
    const uint16_t *params_bf16;    /* [device] BF16 copies, LCS_MLP_BF16 */
} lcs_mlp_t;

/* Bytes of the activation workspace of a batch (training: kept for backward). */
int64_t lcs_mlp_workspace_bytes(int64_t batch, int32_t training);
/* Bytes of the scratch lcs_mlp_backward needs for a batch. */
int64_t lcs_mlp_backward_scratch_bytes(int64_t batch);

/* lcs_mlp_refresh_bf16 -- write the BF16 compute copies of the hidden-layer
 * matrices from the FP32 masters (after initialisation and every update).
 * Errors: LCS_E_ARG, LCS_E_HIP. */
lcs_status lcs_mlp_refresh_bf16(const float *params, uint16_t *params_bf16, void *stream);

/* lcs_mlp_forward -- displacement dx [device] FP32 3 x batch of inputs
 * xt [device] FP32 4 x batch (rows x, y, z, t).  workspace [device] of at least
 * lcs_mlp_workspace_bytes(batch, training) bytes; with training != 0 it keeps
 * the activations lcs_mlp_backward reads.
 * Errors: LCS_E_ARG, LCS_E_SHAPE, LCS_E_HIP. */
lcs_status lcs_mlp_forward(const lcs_mlp_t *mlp, const float *xt, int64_t batch, float *dx,
                           void *workspace, int64_t workspace_bytes, int32_t training,
                           void *stream);

/* lcs_mlp_backward -- grads [device] FP32 LCS_MLP_PARAMS (same layout as the
 * masters) = gradient of sum(ddx * dx) for the batch whose training forward
 * filled `workspace`; ddx [device] FP32 3 x batch.  Gradients are summed over
 * fixed row chunks (2048 rows for hidden weights, 128 for biases and the head)
 * and the chunks in a fixed order (deterministic).  scratch
 * [device] of at least lcs_mlp_backward_scratch_bytes(batch) bytes.
 * Errors: LCS_E_ARG, LCS_E_SHAPE, LCS_E_HIP. */
lcs_status lcs_mlp_backward(const lcs_mlp_t *mlp, const void *workspace, const float *ddx,
                            int64_t batch, float *grads, void *scratch, int64_t scratch_bytes,
                            void *stream);

/* lcs_mse_grad -- mean squared error of pred against target (n values each,
 * [device] FP32): grad = 2 (pred - target) / n (or NULL) and loss [device]
 * FP64 scalar = mean of squares (or NULL), summed in a fixed order.
 * Errors: LCS_E_ARG, LCS_E_SHAPE, LCS_E_HIP. */
lcs_status lcs_mse_grad(const float *pred, const float *target, int64_t n, float *grad,
                        double *loss, void *stream);

/* lcs_adam_step -- one Adam update (Kingma & Ba, bias-corrected; step counts
 * from 1) of params with grads, moment buffers m and v ([device] FP32, n each).
 * Errors: LCS_E_ARG, LCS_E_SHAPE, LCS_E_HIP. */
lcs_status lcs_adam_step(float *params, const float *grads, float *m, float *v, int64_t n,
                         float lr, float beta1, float beta2, float eps, int32_t step,
                         void *stream);

/* lcs_sub -- out = a - b elementwise ([device] FP32, n values each); used to
 * form training displacements xf - x0.  Errors: LCS_E_ARG, LCS_E_SHAPE, LCS_E_HIP. */
lcs_status lcs_sub(const float *a, const float *b, int64_t n, float *out, void *stream);

/* lcs_mlp_train -- n_steps Adam steps of the surrogate on the mean squared
 * error of its displacement (training from trajectories the integrator
 * generated; the local flow-map approximation the paper's Sec. 4 cites).
 * Step s (global, counting from first_step >= 1) trains on batch
 * b = (s - 1) mod floor(n / batch): columns b*batch .. b*batch + batch - 1 of
 * xt [device] FP32 4 x n (rows x, y, z, t; row stride n) and target [device]
 * FP32 3 x n (displacements), with the learning rate decayed along a cosine
 * from lr at step 1 to lr_final at step total_steps, and Adam (Kingma & Ba,
 * bias-corrected) moments m, v [device] FP32, LCS_MLP_PARAMS each.  params and
 * params_bf16 must be the descriptor's own buffers; both are updated after
 * every step.  losses [device] FP64, n_steps values (or NULL): the MSE of each
 * step's batch before its update.  grads [device] FP32 LCS_MLP_PARAMS (or
 * NULL): the last step's gradient.  The rounding points are those of
 * lcs_mlp_forward / lcs_mse_grad / lcs_mlp_backward / lcs_adam_step (BF16
 * operands and activations, FP32 accumulation), but the Fourier features take
 * the hardware sine and cosine of the exactly reduced phase and GELU and its
 * derivative come from one base-2 exponential and reciprocal, so the results
 * agree with those entry points to rounding, not bit for bit; every sum runs
 * in a fixed order, so a call is bit-reproducible.  Four launches per step: forward with the loss
 * gradient, backward through the hidden layers, weight gradients over
 * 2048-sample chunks, and the reduction with Adam and the BF16 copies.
 * workspace [device] of at least lcs_mlp_train_workspace_bytes(batch) bytes
 * (about 6.2 kB per sample).  Nothing is allocated.
 * Errors: LCS_E_ARG, LCS_E_SHAPE, LCS_E_HIP. */
int64_t lcs_mlp_train_workspace_bytes(int64_t batch);
lcs_status lcs_mlp_train(const lcs_mlp_t *mlp, float *params, uint16_t *params_bf16,
                         const float *xt, const float *target, int64_t n, int64_t batch,
                         int32_t first_step, int32_t n_steps, int32_t total_steps, float lr,
                         float lr_final, float beta1, float beta2, float eps, float *m, float *v,
                         double *losses, float *grads, void *workspace, int64_t workspace_bytes,
                         void *stream);

/*
 * Surrogate flow map of a seed grid (3D): composition, check samples, fallback.
 *
 * lcs_surrogate_compose -- x_{k+1} = x_k + dx(x_k, t0 + k tau), k < n_windows,
 *   from the seeds, with the network of `mlp`; xf [device] FP32 3 x Ns.  One
 *   launch: each workgroup keeps 128 seeds' activations in LDS through every
 *   window (features, the four MFMA layers, head, update).
 * lcs_surrogate_check -- check tiles are aligned 16 x 16 x 8 blocks of seeds
 *   (lcs_check_tile_count of them, x fastest); in each, the seeds with local
 *   index 0, 100, 200, ... (about 1 %) are advected with plain RK4 from t0
 *   over T with step dt and compared with xf.  tile_err [device] FP32 = the
 *   largest Euclidean distance in the tile (+inf if a sample was flagged);
 *   tile_fail [device] uint8 = (tile_err > tol); *n_fail [device] int32 = the
 *   number of failing tiles.
 * lcs_advect_tiles -- plain RK4 (as lcs_advect) for every seed of the tiles
 *   with tile_fail != 0, written into xf / cell / flags; other seeds untouched.
 * Errors: LCS_E_ARG, LCS_E_SHAPE, LCS_E_TIME_RANGE, LCS_E_SEED_DOMAIN,
 *   LCS_E_STEP, LCS_E_UNSUPPORTED (2D), LCS_E_HIP.
 */
int64_t lcs_check_tile_count(const lcs_seed_grid_t *seeds);
lcs_status lcs_surrogate_compose(const lcs_mlp_t *mlp, const lcs_seed_grid_t *seeds, double t0,
                                 double tau, int32_t n_windows, float *xf, void *stream);
lcs_status lcs_surrogate_check(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, double t0,
                               double T, double dt, const float *xf, float tol, float *tile_err,
                               uint8_t *tile_fail, int32_t *n_fail, void *stream);
lcs_status lcs_advect_tiles(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, double t0,
                            double T, double dt, const uint8_t *tile_fail, float *xf,
                            int64_t *cell, uint8_t *flags, void *stream);

/*
 * lcs_surrogate_flowmap -- the whole surrogate flow map of a 3D seed grid over
 * T = n_windows * tau (a local flow-map approximation, Sec. 4, with plain RK4
 * as the reference and the fallback): lcs_surrogate_compose, then
 * lcs_surrogate_check with RK4 step dt and tolerance tol, then plain RK4 for
 * the seeds of every failing tile.  When more than whole_grid_fraction of the
 * check tiles fail, the whole grid is re-advected instead with the re-bundled
 * RK4 of lcs_advect_sorted (the same per-tracer arithmetic, so the same
 * results as tile by tile; faster when most tiles fail); whole_grid_fraction
 * >= 1 never takes that branch.  tol = +inf accepts every tile (composition
 * only; the check samples still run and tile_err still reports their error).
 *
 * The call reads the number of failing tiles back to the host: it
 * synchronises `stream` once, after the check, and returns after enqueuing the
 * fallback.
 *
 * xf               [device] FP32, 3 x Ns: composed positions of accepted tiles,
 *                  RK4 positions (bit-identical to lcs_advect) of failing ones.
 * flags            [device] uint8, Ns, or NULL: 0 for seeds of accepted tiles,
 *                  lcs_advect's flags for re-advected seeds.
 * tile_err         [device] FP32, lcs_check_tile_count(seeds), or NULL: the
 *                  per-tile check error (as lcs_surrogate_check).
 * n_fallback_tiles [host] int32 or NULL: number of failing tiles.
 * whole_grid       [host] int32 or NULL: 1 if the whole grid was re-advected.
 * workspace        [device], at least
 *                  lcs_surrogate_flowmap_workspace_bytes(vel, seeds,
 *                  whole_grid_fraction) bytes (per-tile scratch, plus the
 *                  re-bundling workspace when whole_grid_fraction < 1).
 * Errors: LCS_E_ARG (NULL xf / workspace, tol < 0 or NaN, whole_grid_fraction
 *   < 0, n_windows < 1, tau 0), LCS_E_SHAPE (workspace too small), and those
 *   of lcs_surrogate_check; LCS_E_HIP.
 */
int64_t lcs_surrogate_flowmap_workspace_bytes(const lcs_velocity_t *vel,
                                              const lcs_seed_grid_t *seeds,
                                              double whole_grid_fraction);
lcs_status lcs_surrogate_flowmap(const lcs_mlp_t *mlp, const lcs_velocity_t *vel,
                                 const lcs_seed_grid_t *seeds, double t0, double tau,
                                 int32_t n_windows, double tol, double dt,
                                 double whole_grid_fraction, float *xf, uint8_t *flags,
                                 float *tile_err, int32_t *n_fallback_tiles, int32_t *whole_grid,
                                 void *workspace, int64_t workspace_bytes, void *stream);

/*
 * lcs_advect_ab -- as lcs_advect with an explicit Adams-Bashforth multistep
 * method of order 2, 3 or 4 instead of RK4 (Sec. 2 Flow Map filter: single
 * step and multistep methods):
 *   x_{n+1} = x_n + dt * sum_{j<order} b_j u(x_{n-j}, t_{n-j})
 * with b = (3, -1)/2, (23, -16, 5)/12, (55, -59, 37, -9)/24; the first
 * order-1 steps are classical RK4 steps.  One velocity evaluation per step
 * (RK4 takes four).  The exit rule is lcs_advect's, applied to the RK4 stage
 * points of the start-up steps and to every new position.
 * Errors: as lcs_advect, and LCS_E_ARG for an order outside 2..4.
 */
lcs_status lcs_advect_ab(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, int32_t order,
                         double t0, double T, double dt, float *xf, int64_t *cell, uint8_t *flags,
                         void *stream);

/*
 * lcs_advect_ab_sorted -- lcs_advect_ab with the tracers re-bundled by position
 * between segments of segment_steps steps, as lcs_advect_sorted does for RK4
 * (the past velocities travel with each tracer).  Results equal
 * lcs_advect_ab's bit for bit.  workspace: [device], at least
 * lcs_advect_ab_sorted_workspace_bytes(vel, seeds) bytes (valid for every order).
 */
int64_t lcs_advect_ab_sorted_workspace_bytes(const lcs_velocity_t *vel,
                                             const lcs_seed_grid_t *seeds);
lcs_status lcs_advect_ab_sorted(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds,
                                int32_t order, double t0, double T, double dt,
                                int32_t segment_steps, float *xf, int64_t *cell, uint8_t *flags,
                                void *workspace, int64_t workspace_bytes, void *stream);

/*
 * lcs_advect_aux -- flow map of auxiliary points about every seed (Sec. 2
 * Seed filter: highly localised auxiliary points; Cauchy-Green filter: the
 * gradient from differences of auxiliary points).  For every seed x0 and
 * axis b < dim, point q = 2b starts at x0 - delta[b] e_b and point q = 2b+1 at
 * x0 + delta[b] e_b (FP64, carried as two-floats); each is advected exactly as
 * lcs_advect advects a seed (RK4, exit rule, flags).
 *
 * delta   [host] dim doubles > 0 (typically well below the seed spacing).
 * xa_hi,  [device] FP32, each dim x (2*dim) x Ns: component a of point q of
 * xa_lo   seed s at [(a*2*dim + q)*Ns + s]; the final position is
 *         xa_hi + xa_lo (a two-float, exact in FP64).
 * flags   [device] uint8, (2*dim) x Ns, or NULL: [q*Ns + s].
 * Errors: as lcs_advect (seeds must lie in the domain; an auxiliary point
 * that starts outside it is flagged LCS_FLAG_OUT and not moved).
 */
lcs_status lcs_advect_aux(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds,
                          const double *delta, double t0, double T, double dt, float *xa_hi,
                          float *xa_lo, uint8_t *flags, void *stream);

/*
 * lcs_advect_aux_sorted -- lcs_advect_aux with the auxiliary tracers
 * re-bundled by position between segments of segment_steps steps (0: 50), as
 * lcs_advect_sorted does for seeds.  Same outputs, bit for bit.
 * workspace [device], at least lcs_advect_aux_sorted_workspace_bytes(vel, seeds)
 * bytes (caller-owned).  Errors: as lcs_advect_aux and lcs_advect_sorted, and
 * LCS_E_SHAPE for more than 2^31-1 auxiliary points.
 */
int64_t lcs_advect_aux_sorted_workspace_bytes(const lcs_velocity_t *vel,
                                              const lcs_seed_grid_t *seeds);
lcs_status lcs_advect_aux_sorted(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds,
                                 const double *delta, double t0, double T, double dt,
                                 int32_t segment_steps, float *xa_hi, float *xa_lo, uint8_t *flags,
                                 void *workspace, int64_t workspace_bytes, void *stream);

/*
 * lcs_cg_aux -- Cauchy-Green tensor from auxiliary points (Eq. 1; Sec. 2
 * Cauchy-Green filter): J[a][b] = (F_a(x0 + delta_b e_b) - F_a(x0 - delta_b e_b))
 * / (2 delta_b) in FP64 from the exact two-float positions, C = J^T J packed as
 * lcs_cg_tensor.  stencil_flags (or NULL) gets LCS_FLAG_STENCIL_OUT where a
 * point of the seed is flagged (flags may be NULL).
 */
lcs_status lcs_cg_aux(const lcs_seed_grid_t *seeds, const double *delta, const float *xa_hi,
                      const float *xa_lo, const uint8_t *flags, double *C, uint8_t *stencil_flags,
                      void *stream);

/*
 * lcs_cg_eig -- eigenvalues and eigenvectors of the packed symmetric tensors
 * C (Sec. 2 Cauchy-Green filter: eigenvalue and eigenvector fields for LCS
 * detection), FP64 cyclic Jacobi per point.
 * C       [device] FP64, (dim(dim+1)/2) x n, packed as lcs_cg_tensor writes it.
 * evals   [device] FP64, dim x n, ascending: evals[k*n + p]; or NULL.
 * evecs   [device] FP64, dim x dim x n: component a of the eigenvector of
 *         evals[k] at [(k*dim + a)*n + p], unit length, signed so that its
 *         largest component is positive; or NULL.
 */
lcs_status lcs_cg_eig(int32_t dim, int64_t n, const double *C, double *evals, double *evecs,
                      void *stream);

/*
 * lcs_advect_snapshots -- the flow map at several times of one integration
 * (Sec. 3.1: the CG tensor can be evaluated at any step; Sec. 4: the CG
 * tensor at various integration times).  As lcs_advect from t0 with step dt
 * (no periodic-domain restriction beyond lcs_advect's), recording every tracer
 * after each of the n_snap step counts snap_steps[k] (host, strictly
 * increasing, >= 1, 1 <= n_snap <= LCS_MAX_SNAPSHOTS); the interval
 * [t0, t0 + snap_steps[n_snap-1]*dt] must lie in the frame span.
 * xf          [device] FP32, n_snap x dim x Ns: [(k*dim + a)*Ns + s]; a tracer
 *             frozen earlier keeps its frozen position.
 * flags       [device] uint8, n_snap x Ns, or NULL: the flag as of snapshot k.
 * steps_done  [device] int32, Ns, or NULL: steps taken before the tracer froze
 *             (snap_steps[n_snap-1] if it never did).
 * The FTLE at snapshot k is lcs_cg_ftle on xf + k*dim*Ns with
 * T = snap_steps[k]*dt.
 */
lcs_status lcs_advect_snapshots(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, double t0,
                                double dt, int32_t n_snap, const int32_t *snap_steps, float *xf,
                                uint8_t *flags, int32_t *steps_done, void *stream);

/* Workspace of lcs_ftle_early for seeds: room for every seed at once (smaller
 * workspaces process the listed seeds in chunks). */
int64_t lcs_ftle_early_workspace_bytes(const lcs_seed_grid_t *seeds);

/*
 * lcs_ftle_early -- FTLE with early evaluation (Sec. 2 Flow Map filter: when a
 * trajectory leaves the domain, the CG tensor is evaluated early at every
 * location that relies on it).  For seed s, n_s = the smallest steps_done over
 * the seeds its gradient uses (itself and its grid neighbours as
 * lcs_cg_tensor differences them).  n_s = nsteps: the ordinary FTLE from xf.
 * 0 < n_s < nsteps: its stencil is re-advected n_s steps from t0 and
 * sigma = ln(lambda_max) / (2 n_s |dt|).  n_s = 0: NaN.
 * xf          [device] FP32, dim x Ns: positions after nsteps (lcs_advect or
 *             the last snapshot).
 * steps_done  [device] int32, Ns (lcs_advect_snapshots).
 * lambda_max  [device] FP64, Ns, or NULL.  ftle [device] FP64, Ns.
 * t_eff       [device] FP64, Ns, or NULL: n_s * dt.
 * workspace   [device], >= 8*Ns + 2048 bytes (lcs_ftle_early_workspace_bytes
 *             for a single pass).
 * Synchronises the stream (the number of listed seeds decides the passes).
 */
lcs_status lcs_ftle_early(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, double t0,
                          double dt, int32_t nsteps, const float *xf, const int32_t *steps_done,
                          double *lambda_max, double *ftle, double *t_eff, void *workspace,
                          int64_t workspace_bytes, void *stream);

/* ======================================================================== */
/* Unstructured velocity data: triangle (2D) and tetrahedron (3D) meshes      */
/* ======================================================================== */
/*
 * Sec. 3.2: unstructured velocity data is tetrahedralised (triangulated in
 * 2D) so that one cell search and one interpolation kernel serve every grid
 * topology; the cell holding a point is found by a local search that starts
 * from the cell that held the tracer before.  Inside a cell the velocity is
 * the piecewise-linear interpolant sum_i lambda_i u(node_i), lambda the
 * barycentric coordinates of the point; in time it is linear between the two
 * frames that bracket t, as on structured grids.
 *
 * Local search: from a start cell, compute the barycentric coordinates of the
 * point; if the smallest is >= -LCS_MESH_EPS the point is in that cell,
 * otherwise step to the neighbour across the face opposite the vertex with the
 * smallest coordinate.  Reaching a boundary face means the point is outside
 * the mesh (LCS_FLAG_OUT); more than LCS_MESH_MAX_WALK steps set
 * LCS_FLAG_LOST.  A point's first cell comes from a uniform grid of buckets
 * over the mesh's bounding box, each holding one cell near it.
 */

/* Containment tolerance on barycentric coordinates and step limit of the
 * local cell search. */
#define LCS_MESH_EPS 3.814697265625e-06 /* 2^-18 */
#define LCS_MESH_MAX_WALK 1024

/*
 * Mesh description, read by lcs_mesh_create only.
 *
 * dim      2 (triangles) or 3 (tetrahedra).
 * n_nodes  1 <= n_nodes < 2^28.   n_cells  1 <= n_cells < 2^31.
 * nodes    [device] FP64, [n_nodes][dim] node coordinates (x fastest).
 * cells    [device] int32, [n_cells][dim+1] node ids of each cell, any
 *          vertex order.  The mesh must be conforming: a face is shared by at
 *          most two cells, and no cell is degenerate.
 */
typedef struct {
    int32_t dim;
    int32_t reserved;         /* must be 0 */
    int64_t n_nodes;
    int64_t n_cells;
    const double *nodes;
    const int32_t *cells;
} lcs_mesh_desc_t;

/* Opaque mesh: the library's device copy of the cell geometry (the affine
 * map of every cell to barycentric coordinates, FP32), the node ids and face
 * neighbours of every cell, and the bucket grid for first location. */
typedef struct lcs_mesh *lcs_mesh_t;

/* Mesh facts (host struct filled by lcs_mesh_info). */
typedef struct {
    int32_t dim;
    int32_t reserved;
    int64_t n_nodes;
    int64_t n_cells;
    int64_t n_boundary_faces; /* faces with no neighbouring cell */
    int64_t buckets[3];       /* bucket grid of the first-location search */
    double lo[3], hi[3];      /* bounding box of the nodes */
    int64_t device_bytes;     /* device memory the mesh object holds */
} lcs_mesh_info_t;

/*
 * Velocity at the mesh nodes for a series of frames (Sec. 2 Interpolator:
 * frames resident in GPU memory).
 *
 * n_frames  >= 2; frame f holds the field at t_first + f*dt_frame,
 *           dt_frame > 0.
 * u         [device] FP32, [n_frames][n_nodes][S] with S = 2 in 2D and S = 4
 *           in 3D (x, y, z and one unused value): the components of a node
 *           sit together so that one 8- or 16-byte load reads them.
 */
typedef struct {
    int32_t n_frames;
    int32_t reserved;         /* must be 0 */
    double t_first;
    double dt_frame;
    const float *u;
} lcs_mesh_frames_t;

/*
 * lcs_mesh_create -- build the device mesh object (Sec. 2 Seed and Reader
 * filters: a one-time preparation of the velocity mesh).  Computes, on the
 * device, the face neighbours of every cell (through a node-to-cell adjacency
 * list), every cell's affine map to barycentric coordinates (in FP64, stored
 * as FP32 relative to an FP32 reference point with an FP64-exact offset) and
 * the bucket grid.  Allocates device memory owned by the mesh object and
 * synchronises the stream before it returns.
 * Errors: LCS_E_ARG (NULL, dim), LCS_E_SHAPE (counts, a node id out of range,
 * a degenerate cell, a face shared by more than two cells), LCS_E_HIP.
 */
lcs_status lcs_mesh_create(const lcs_mesh_desc_t *desc, lcs_mesh_t *out, void *stream);

/* lcs_mesh_destroy -- frees the mesh object (NULL is ignored); waits for the
 * device first. */
void lcs_mesh_destroy(lcs_mesh_t mesh);

/* lcs_mesh_info -- facts about a mesh object.  info: [host]. */
lcs_status lcs_mesh_info(lcs_mesh_t mesh, lcs_mesh_info_t *info);

/*
 * lcs_mesh_locate -- cell holding each point (first location: bucket start
 * cell, then the local search).
 * x     [device] FP32, dim x n.
 * cell  [device] int64, n: cell id, -1 outside the mesh (or non-finite x),
 *       -2 if the search hit its step limit.
 * lam   [device] FP32, (dim+1) x n, or NULL: barycentric coordinates in that
 *       cell (unspecified where cell < 0).
 */
lcs_status lcs_mesh_locate(lcs_mesh_t mesh, const float *x, int64_t n, int64_t *cell, float *lam,
                           void *stream);

/*
 * lcs_mesh_velocity_at -- u(x, t) at points, each with its own time (Sec. 3.2:
 * cell search, then piecewise-linear interpolation in space and linear in
 * time).  A time outside the frame span is clamped to it (the values are not
 * read on the host, so no error is reported for them).
 * x [device] FP32 dim x n; t [device] FP64 n; u [device] FP32 dim x n (NaN
 * outside the mesh); cell [device] int64 n or NULL (as lcs_mesh_locate).
 */
lcs_status lcs_mesh_velocity_at(lcs_mesh_t mesh, const lcs_mesh_frames_t *frames, const float *x,
                                const double *t, int64_t n, float *u, int64_t *cell, void *stream);

/*
 * lcs_mesh_advect -- flow map of a structured seed grid through velocity on a
 * mesh (Eq. 2; Sec. 2 Seed and Flow Map filters; Sec. 3.1 RK4; Sec. 3.2 local
 * cell search).  N = T/dt classical RK4 steps, t_n = t0 + n*dt; the four
 * stage points and the new position are located by the local search started
 * from the cell of the previous one, so each tracer carries its cell from step
 * to step.  A seed outside the mesh is flagged LCS_FLAG_OUT and not moved (an
 * unstructured domain rarely fills the seed grid's box).  A stage point or new
 * position outside the mesh rejects the step and freezes the tracer
 * (LCS_FLAG_OUT), as do non-finite values (LCS_FLAG_NONFINITE) and a search
 * past its step limit (LCS_FLAG_LOST).
 *
 * seeds  non-periodic seed grid of the mesh's dim (else LCS_E_UNSUPPORTED /
 *        LCS_E_ARG).
 * xf     [device] FP32, dim x Ns, final positions.
 * cell   [device] int64, Ns, or NULL: mesh cell holding the final position
 *        (-1 for a seed outside the mesh).
 * flags  [device] uint8, Ns, or NULL.
 * Errors: LCS_E_ARG, LCS_E_TIME_RANGE, LCS_E_STEP, LCS_E_HIP.
 */
lcs_status lcs_mesh_advect(lcs_mesh_t mesh, const lcs_mesh_frames_t *frames,
                           const lcs_seed_grid_t *seeds, double t0, double T, double dt,
                           float *xf, int64_t *cell, uint8_t *flags, void *stream);

/*
 * lcs_mesh_advect_points -- as lcs_mesh_advect for arbitrary points x0
 * ([device] FP32 dim x n) with their own start times t0 ([device] FP64 n);
 * a point whose interval [t0, t0+T] leaves the frame span is not moved and is
 * flagged LCS_FLAG_TIME_OUT.  n = 0 does nothing (after the mesh, frames and
 * step count are validated); n must stay below 2^31.
 */
lcs_status lcs_mesh_advect_points(lcs_mesh_t mesh, const lcs_mesh_frames_t *frames,
                                  const float *x0, const double *t0, int64_t n, double T,
                                  double dt, float *xf, int64_t *cell, uint8_t *flags,
                                  void *stream);

/*
 * lcs_timing_enable / lcs_timing_query -- measurement of the library's main
 * kernels (not part of the method).  While timing is enabled, every launch of
 * advect_grid_kernel<D>, rebundle_segment_kernel<D, S>, cg_kernel<D, fused>,
 * compose_fused_kernel, gemm_kernel<EPI_FWD|EPI_BWD> and wgrad_kernel is
 * bracketed by two HIP events recorded on the stream the kernel is launched
 * on (two event creations and records per launch).  lcs_timing_enable(on)
 * discards earlier records and turns recording on (on != 0) or off.
 * lcs_timing_query(kernel, launches, total_ms) -- after the recorded work has
 * completed (synchronise first) -- gives the number of recorded launches of
 * the kernel named exactly as above (e.g. "rebundle_segment_kernel<3, 0>") and
 * their summed duration in milliseconds.  Thread safe; records are global to
 * the process.  Errors: LCS_E_ARG (NULL pointer), LCS_E_HIP (work not done).
 */
lcs_status lcs_timing_enable(int32_t on);
lcs_status lcs_timing_query(const char *kernel, int64_t *launches, double *total_ms);

/* lcs_sync_status -- waits for the stream and reports a pending HIP error. */
lcs_status lcs_sync_status(void *stream);

/* lcs_last_error -- thread-local text for the last non-OK status ("" if none). */
const char *lcs_last_error(void);

/* lcs_version -- library ABI version (major*10000 + minor*100 + patch). */
int32_t lcs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LCS_H */
