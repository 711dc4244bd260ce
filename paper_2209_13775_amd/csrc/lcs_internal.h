// lcs_internal.h -- device-side parameter blocks and launcher prototypes
// shared by the HIP translation units of the library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lcs.h"

namespace lcs {

constexpr int kWave = 64;   // CDNA wavefront width

// Velocity frames as the kernels read them.  FP32 copies of the geometry
// drive the FP32 advection; the FP64 copies are used only for the FP64 cell
// index of the returned positions.
struct VelDev {
    const float *u[3];        // structure-of-arrays components (ilv == 0)
    const float *ilv_u;       // interleaved frames (ilv = floats per node: 2, 3 or 4)
    int ilv;
    long long frame_stride;   // n0*n1*n2
    uint32_t sb[3];           // bytes between nodes adjacent along each axis, within one
                              // frame array (every offset in a frame fits 32 bits)
    int n[3];
    float nf[3];
    float oh[3], ol[3];       // origin as a two-float (hi + lo)
    float ih[3], il[3];       // 1/spacing as a two-float (hi + lo)
    float lo[3], hi[3];       // closed domain on non-periodic axes
    uint32_t periodic_mask;
    int n_frames;
    double t_first;
    double dt_frame;
    double inv_dt_frame;
    double origin_d[3];
    double spacing_d[3];
    double t_last;            // t_first + (n_frames-1)*dt_frame
};

// Work decomposition of a structured seed grid: the grid is cut into
// workgroup tiles (waves_per_axis x wave_tile seeds) and the tiles are visited
// along a Morton (Z-order) curve; consecutive workgroups on one XCD take
// consecutive curve positions.
struct SeedTiling {
    int sn[3];                // seeds per axis
    double s_origin[3];
    double s_spacing[3];
    int wt[3];                // wave sub-tile (product 64)
    int wg[3];                // waves per workgroup along each axis
    int ntiles[3];            // workgroup tiles per axis
    int bits[3];              // Morton bits per axis (ceil log2 ntiles)
    int max_bits;
    int n_blocks;             // launched workgroups (Morton index space)
};

struct AdvectArgs {
    VelDev v;
    SeedTiling g;
    double t0, dt;
    int nsteps;
    long long ns;             // number of tracers
    float *xf;
    long long *cell;
    uint8_t *flags;
    // points mode
    const float *x0;
    const double *t0v;
    double T;
};

struct CgArgs {
    int dim;
    int n[3];
    uint32_t periodic_mask;
    double h[3];
    double period[3];
    long long ns;
    const float *xf;
    const uint8_t *flags;
    double *C;                // may be null (fused mode)
    uint8_t *sflags;
    double *lam;
    double *ftle;
    double inv_two_T;         // 1 / (2|T|)
};

// Auxiliary-point advection: the seed tiling of `a` times 2*dim points.
struct AuxArgs {
    AdvectArgs a;
    double delta[3];
    float *xa_hi;             // [dim][2*dim][Ns]
    float *xa_lo;
};

struct CgAuxArgs {
    int dim;
    long long ns;
    double delta[3];
    const float *xa_hi;
    const float *xa_lo;
    const uint8_t *flags;     // [2*dim][Ns] or null
    double *C;
    uint8_t *sflags;
};

// Time-resolved flow map: positions after each listed step count.
constexpr int kMaxSnapshots = LCS_MAX_SNAPSHOTS;

struct SnapArgs {
    AdvectArgs a;
    int n_snap;
    int steps[kMaxSnapshots];  // strictly increasing, >= 1
    float *xf;                 // [n_snap][dim][Ns]
    uint8_t *flags;            // [n_snap][Ns] or null
    int *steps_done;           // [Ns] or null
};

// Early Cauchy-Green evaluation (list of seeds whose stencil left the domain).
struct EarlyArgs {
    int dim;
    int n[3];
    uint32_t periodic_mask;
    double h[3];
    long long ns;
    int nsteps;
    double dt;
    const float *xf;           // [dim][Ns] after nsteps
    const int *steps_done;     // [Ns]
    double *lam;               // may be null
    double *ftle;
    double *t_eff;             // may be null
    int *counter;
    int *list;                 // [2*Ns]: (seed, n_s)
    double *pos;               // [chunk][7][3] re-advected stencil positions
};

struct EarlyAdvArgs {
    VelDev v;
    double s_origin[3];
    double s_spacing[3];
    int n[3];
    uint32_t periodic_mask;
    double t0, dt;
    const int *list;
    double *pos;
};

struct FtleArgs {
    long long n;
    const double *C;
    double *lam;
    double *ftle;
    double inv_two_T;
};

// Batched windows: (window, tile) work items, windows sorted by step count
// (longest first) and claimed through an atomic counter by persistent blocks.
constexpr int kMaxWindows = LCS_MAX_WINDOWS;

struct WindowDev {
    double t0;
    int nsteps;
    int out_index;            // position of the window in the caller's order
};

// Persistent batched advection: one work counter per XCD (blocks are dealt
// round-robin to the 8 XCDs, so block b runs on XCD b % 8).
constexpr int kBatchCounters = 8;

struct BatchArgs {
    VelDev v;
    SeedTiling g;
    double dt;
    long long ns;
    int n_windows;
    int total_items;          // n_windows * g.n_blocks
    int *counter;             // kBatchCounters work counters (device), one per XCD
    float *xf;
    long long *cell;
    uint8_t *flags;
    WindowDev win[kMaxWindows];
};

static_assert(sizeof(BatchArgs) <= 4096, "kernel arguments must fit the 4 KiB kernarg segment");

// ---------------------------------------------------------------------------
// Fourier-feature MLP surrogate (fixed architecture: 64 frequencies -> 128
// features -> 4 x 256 GELU -> 3)
// ---------------------------------------------------------------------------
constexpr int kMlpFreq = LCS_MLP_FREQ;
constexpr int kMlpFeat = 2 * LCS_MLP_FREQ;
constexpr int kMlpWidth = LCS_MLP_WIDTH;
constexpr int kMlpHidden = LCS_MLP_HIDDEN;
constexpr long long kMlpParams = LCS_MLP_PARAMS;
constexpr long long kBf16Count = LCS_MLP_BF16;
constexpr int kHeadPart = 3 * kMlpWidth + 3;

__host__ __device__ constexpr int mlp_in_width(int l) { return l == 0 ? kMlpFeat : kMlpWidth; }
// FP32 parameter offsets: W_l ([in][out], row-major) then b_l, for l = 0..3; then W_h, b_h
__host__ __device__ constexpr long long mlp_off_w(int l)
{
    return l == 0 ? 0 : (long long)kMlpFeat * kMlpWidth + kMlpWidth +
                            (long long)(l - 1) * ((long long)kMlpWidth * kMlpWidth + kMlpWidth);
}
__host__ __device__ constexpr long long mlp_off_b(int l)
{
    return mlp_off_w(l) + (long long)mlp_in_width(l) * kMlpWidth;
}
constexpr long long kOffWh = mlp_off_w(kMlpHidden);
constexpr long long kOffBh = kOffWh + 3LL * kMlpWidth;
static_assert(kOffBh + 3 == kMlpParams, "parameter layout");
// BF16 copies: for each hidden layer, W_l ([in][out]) then W_l^T ([out][in]),
// both in fragment order (frag_index)
__host__ __device__ constexpr long long mlp_off_bf16(int l)
{
    return l == 0 ? 0 : mlp_off_bf16(l - 1) + 2LL * mlp_in_width(l - 1) * kMlpWidth;
}
static_assert(mlp_off_bf16(kMlpHidden) == kBf16Count, "bf16 layout");

struct MlpDev {
    const float *freq;
    float in_shift[4];
    float in_scale[4];
    float out_scale;
    const float *params;
    const uint16_t *wbf;
};

// Element (n, k) of an N x K BF16 matrix kept in MFMA fragment order: blocks
// of 16 rows x 32 columns (K/32 blocks per block row, block rows in order),
// each 64 lanes x 8 values, lane (n % 16) + 16 ((k % 32) / 8) holding the 8
// consecutive k of its row -- so a wave's A-operand fragment of a block is one
// contiguous 1 KiB.  N % 16 == 0 and K % 32 == 0.
__host__ __device__ constexpr long long frag_index(int n, int k, int K)
{
    return ((long long)(n / 16) * (K / 32) + k / 32) * 512 + ((n % 16) + 16 * ((k % 32) / 8)) * 8 + k % 8;
}

struct GemmArgs {
    const uint16_t *A;        // [M][K]
    const uint16_t *Bt;       // [N][K], row-major or (bt_frag) in fragment order
    long long M;
    int N, K;
    const float *bias;        // forward only
    uint16_t *H;              // output [M][N]
    uint16_t *Z;              // forward: pre-activation out (optional); backward: pre-activation in
    int bt_frag;              // Bt in fragment order (frag_index)
};

struct WgradArgs {
    const uint16_t *X;        // [M][K]
    const uint16_t *D;        // [M][N]
    long long M;
    int K, N;
    long long chunk;
    float *part;              // [nchunk][K][N]
};

struct AdamArgs {
    float lr, beta1, beta2, eps, c1, c2;
};

hipError_t launch_features(const MlpDev &P, const float *xt, long long M, uint16_t *H0, hipStream_t s);
hipError_t launch_gemm(const GemmArgs &g, bool backward, hipStream_t s);
hipError_t launch_wgrad(const WgradArgs &g, int nchunk, hipStream_t s);
hipError_t launch_colsum(const uint16_t *D, long long M, int N, long long chunk, int nchunk,
                         float *part, hipStream_t s);
hipError_t launch_reduce_chunks(const float *part, int nchunk, long long len, float *out, hipStream_t s);
hipError_t launch_head_fwd(const MlpDev &P, const uint16_t *H4, long long M, float *dx, hipStream_t s);
hipError_t launch_head_bwd(const MlpDev &P, const float *ddx, const uint16_t *Z4, const uint16_t *H4,
                           long long M, uint16_t *dZ4, long long chunk, int nchunk, float *part,
                           hipStream_t s);
hipError_t launch_mse(const float *pred, const float *target, long long n, float scale, float *grad,
                      double *loss, double loss_mult, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, long long n, const AdamArgs &a,
                       hipStream_t s);
hipError_t launch_refresh_bf16(const float *params, uint16_t *out, hipStream_t s);

// Fused training step (train.hip): forward + MSE gradient, backward-data,
// weight gradients, then fixed-order reduction + Adam + BF16 copies.
constexpr long long kWgradChunk = 2048;   // samples per weight-gradient partial (multiple of 128)
struct TrainArgs {
    MlpDev P;
    const float *xt;          // [4][ld] inputs of the batch (already offset to its first sample)
    const float *target;      // [3][ld] target displacements
    long long ld;             // row stride of xt and target
    long long B, Bp;          // samples, samples padded to whole 128-sample tiles
    long long n_tiles, n_chunks;
    float mse_scale;          // 2 / (3 B)
    double loss_mult;         // 1 / (3 B)
    uint16_t *dgelu[kMlpHidden];   // gelu'(z_l), fragment layout
    uint16_t *ht[kMlpHidden];      // layer inputs h_l, T8 layout
    uint16_t *dzt[kMlpHidden];     // dz_l, T8 layout
    float *dy;                // [3][Bp] gradient at the head output
    float *part_head;         // [n_tiles][kHeadPart]
    double *part_loss;        // [n_tiles]
    float *part_w;            // [n_chunks][kMlpParams] gradient partials per sample chunk
    float *pred;              // optional [3][B] predictions
    float *params;            // FP32 masters (updated in place; = P.params)
    uint16_t *wbf;            // BF16 copies (updated; = P.wbf)
    float *m, *v;             // Adam moments
    float *grads;             // optional: the step's gradient
    double *loss;             // optional: the step's MSE
};
hipError_t launch_train_step(const TrainArgs &a, const AdamArgs &ad, hipStream_t s);

// Surrogate check samples (3D): tiles of 16 x 16 x 8 seeds.
constexpr int kCheckTile[3] = {16, 16, 8};

struct CheckArgs {
    VelDev v;
    SeedTiling g;             // only sn, s_origin, s_spacing are used
    double t0, dt;
    int nsteps;
    long long ns;
    const float *xf;          // surrogate positions, 3 x ns
    float *tile_err;          // per check tile
    long long n_tiles;
    int ct[3];                // check tiles per axis
};

hipError_t launch_surrogate_check(const CheckArgs &a, float tol, uint8_t *tile_fail, int *n_fail,
                                  hipStream_t s);
hipError_t launch_advect_tiles(const AdvectArgs &a, const uint8_t *tile_fail, int ct0, int ct1,
                               long long n_tiles, hipStream_t s);
struct ComposeArgs {
    MlpDev P;
    SeedTiling g;             // sn, s_origin, s_spacing
    long long ns;
    double t0, tau;
    int n_windows;
    float *xf;
};
hipError_t launch_compose_fused(const ComposeArgs &a, hipStream_t s);
hipError_t launch_sub(const float *a, const float *b, long long n, float *out, hipStream_t s);

// ---------------------------------------------------------------------------
// Re-bundled advection: the integration runs in segments; after each segment
// the tracers are counting-sorted by the Morton code of the coarse cell (2^D
// velocity cells) they occupy, so that the lanes of a wave gather from one
// compact region again.  State is carried in HBM between segments.
// ---------------------------------------------------------------------------
constexpr int kMaxBinKeyBits = 24;   // sort bins are one cell wide while their Morton keys fit
                                     // in this many bits (else 2, 4, ... cells wide)

struct TracerState {
    float *xh[3];
    float *xl[3];
    int *idx;                         // seed index (natural order)
    uint8_t *flag;
    float *hist[9];                   // multistep: past velocities [j*dim + a] (null for RK4)
};

struct SortKeys {
    int bits[3];                      // Morton bits per axis
    int max_bits;
    int nb[3];                        // bins per axis
    float inv_bin[3];                 // 1 / (bin width)
    float origin[3];
    uint32_t *keys;                   // [N]
    uint32_t *counts;                 // [n_keys]; turned into offsets by the scan
    uint32_t *block_sums;             // scan scratch
    uint32_t *perm;                   // [N]: sorted slot -> slot of the state it reads
    uint32_t *rank;                   // [N]: slot's place among the slots of its key (histogram)
    long long n_keys;
};

struct SegmentArgs {
    VelDev v;
    SeedTiling g;
    double t0, dt;
    int n_begin, n_end;
    long long n;                      // tracers
    TracerState st;                   // state read (slot sk.perm[p] for slot p)
    TracerState out;                  // state written (slot p)
    SortKeys sk;
    int last;                         // 1: write outputs instead of state + keys
    int order;                        // 0: RK4; 2..4: Adams-Bashforth
    float *xf;
    float *xf_lo;                     // non-null: xf gets the high and xf_lo the low part
    long long *cell;
    uint8_t *flags;
    int aux;                          // tracer q*ns_seeds + s: auxiliary point q of seed s
    long long ns_seeds;
    double delta[3];
};

hipError_t launch_rebundle_init(int dim, const SegmentArgs &a, hipStream_t s);
hipError_t launch_rebundle_segment(int dim, const SegmentArgs &a, hipStream_t s);
hipError_t launch_rebundle_sort(const SegmentArgs &a, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, long long n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, long long n, uint8_t v, hipStream_t s);
long long exclusive_scan_sums_needed(long long n);
hipError_t launch_exclusive_scan_u32(uint32_t *data, long long n, uint32_t *block_sums,
                                     hipStream_t s);

// host-side validation and descriptor conversion (api.hip)
lcs_status validate_velocity(const lcs_velocity_t *v);
lcs_status validate_seeds(const lcs_seed_grid_t *g, int dim);
lcs_status validate_steps(double T, double dt, int *nsteps);
lcs_status validate_seed_domain(const lcs_velocity_t *v, const lcs_seed_grid_t *g);
VelDev velocity_dev(const lcs_velocity_t *v);
SeedTiling seed_tiling(const lcs_seed_grid_t *g);

// Launch timing (lcs_timing_enable): while enabled, a LaunchTimer brackets a
// kernel launch with two HIP events recorded on the launch's stream, filed
// under the kernel's name; disabled, it does nothing.
struct LaunchTimer {
    int slot = -1;
    LaunchTimer(const char *name, hipStream_t s);
    void stop(hipStream_t s);
};

// error reporting shared by the ABI translation units
lcs_status set_error(lcs_status st, const char *fmt, ...);
lcs_status clear_error();
lcs_status hip_error(hipError_t e, const char *where);

hipError_t launch_advect_grid(int dim, const AdvectArgs &a, hipStream_t s);
hipError_t launch_interleave(int dim, int S, const float *const *u, long long nodes, int f_count,
                             long long f_first, float *out, hipStream_t s);
hipError_t launch_interleave_tpair(int dim, const float *const *u, const int *n, int f_count, int f_first,
                                 float *out, hipStream_t s);
hipError_t launch_advect_ab(int dim, int order, const AdvectArgs &a, hipStream_t s);
hipError_t launch_advect_aux(int dim, const AuxArgs &a, hipStream_t s);
hipError_t launch_advect_snap(int dim, const SnapArgs &a, hipStream_t s);
hipError_t launch_early_advect(int dim, const EarlyAdvArgs &a, int first, int count, hipStream_t s);
hipError_t launch_early_mark(const EarlyArgs &a, hipStream_t s);
hipError_t launch_early_cg(const EarlyArgs &a, int first, int count, hipStream_t s);
hipError_t launch_eig(int dim, long long n, const double *C, double *evals, double *evecs,
                      hipStream_t s);
hipError_t launch_cg_aux(const CgAuxArgs &a, hipStream_t s);
hipError_t launch_reset_counter(int *counter, hipStream_t s);
hipError_t launch_advect_batched(int dim, const BatchArgs &a, int grid_blocks, hipStream_t s);
int batched_blocks_per_cu(int dim);
hipError_t launch_advect_points(int dim, const AdvectArgs &a, hipStream_t s);
hipError_t launch_cg(const CgArgs &a, bool fused, hipStream_t s);
hipError_t launch_ftle(int dim, const FtleArgs &a, hipStream_t s);

// ---------------------------------------------------------------------------
// Unstructured meshes (triangles / tetrahedra)
// ---------------------------------------------------------------------------
// Per-cell affine map to barycentric coordinates, relative to an FP32
// reference point r (the FP32 rounding of vertex 0) with an offset c that
// carries the FP64 difference r - v0:
//   lambda_{k+1} = M_k . (x - r) + c_k  (k < dim),  lambda_0 = 1 - sum_k lambda_{k+1}.
// 3D, 4 float4 per cell: (r.xyz, c0), (M0.xyz, c1), (M1.xyz, c2), (M2.xyz, 0)
// 2D, 2 float4 per cell: (r.xy, c0, c1), (M0.xy, M1.xy)
// Per cell one record of RS float4 (96 B in 3D, 64 B in 2D): G float4 of
// geometry, the face neighbours (int4, -1 on a boundary face; neighbour i is
// across the face opposite vertex i), the node ids (int4, .w = -1 in 2D), so
// a walk step and an evaluation's node ids come from the lines the geometry
// load brought in.  (Padding 3D records to 128 B measured slower: the larger
// footprint costs more than the alignment gains.)
template <int D> struct MeshGeo {
    static constexpr int G = (D == 3) ? 4 : 2;
    static constexpr int RS = (D == 3) ? 6 : 4;
    static constexpr int NBR = G, CONN = G + 1;
};

struct MeshDev {
    const float4 *rec;        // [n_cells][RS] cell records
    const int *loc;           // [nb0*nb1*nb2] first-location start cell per bucket (-1 none)
    int nb[3];
    float lo[3];
    float inv_bs[3];
    float eps;
    int max_walk;
};

struct MeshFramesDev {
    const float *u;           // [n_frames][n_nodes][S]
    long long frame_stride;   // n_nodes * S floats
    int n_frames;
    double t_first;
    double inv_dt_frame;
    double t_last;
};

struct MeshAdvectArgs {
    MeshDev m;
    MeshFramesDev f;
    SeedTiling g;             // seed-grid mode
    double t0, dt;
    int nsteps;
    long long ns;
    float *xf;
    long long *cell;
    uint8_t *flags;
    const float *x0;          // points mode
    const double *t0v;
    double T;
};

struct MeshLocGrid {          // bucket grid in FP64 (built once)
    double lo[3];
    double bs[3];
    int nb[3];
};

// mesh preparation (error bits: 1 node id out of range, 2 degenerate cell,
// 4 face shared by more than two cells)
hipError_t launch_mesh_degree(int dim, const int32_t *cells, long long n_cells, long long n_nodes,
                              uint32_t *deg, int *err, hipStream_t s);
hipError_t launch_mesh_adjacency(int dim, const int32_t *cells, long long n_cells,
                                 long long n_nodes, uint32_t *off, int32_t *adj, hipStream_t s);
hipError_t launch_mesh_cells(int dim, const double *nodes, const int32_t *cells, long long n_cells,
                             const uint32_t *off, const int32_t *adj, float4 *rec, int *err,
                             unsigned long long *n_boundary, hipStream_t s);
hipError_t launch_mesh_bbox(int dim, const double *nodes, long long n_nodes, double *part,
                            int n_parts, double *out, hipStream_t s);
hipError_t launch_mesh_raster(int dim, const double *nodes, const int32_t *cells, long long n_cells,
                              const MeshLocGrid &g, int *contain, int *touch, hipStream_t s);
hipError_t launch_mesh_locator_finish(const int *contain, const int *touch, long long n,
                                      int *loc, hipStream_t s);
// queries and advection
hipError_t launch_mesh_locate(int dim, const MeshDev &m, const float *x, long long n,
                              long long *cell, float *lam, hipStream_t s);
hipError_t launch_mesh_velocity(int dim, const MeshDev &m, const MeshFramesDev &f, const float *x,
                                const double *t, long long n, float *u, long long *cell,
                                hipStream_t s);
hipError_t launch_mesh_advect(int dim, const MeshAdvectArgs &a, hipStream_t s);
hipError_t launch_mesh_advect_points(int dim, const MeshAdvectArgs &a, hipStream_t s);

}  // namespace lcs
