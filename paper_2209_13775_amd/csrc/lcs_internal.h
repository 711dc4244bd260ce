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
    const float *u[3];
    long long frame_stride;   // n0*n1*n2
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

struct BatchArgs {
    VelDev v;
    SeedTiling g;
    double dt;
    long long ns;
    int n_windows;
    int total_items;          // n_windows * g.n_blocks
    int *counter;             // work counter (device)
    float *xf;
    long long *cell;
    uint8_t *flags;
    WindowDev win[kMaxWindows];
};

static_assert(sizeof(BatchArgs) <= 4096, "kernel arguments must fit the 4 KiB kernarg segment");

hipError_t launch_advect_grid(int dim, const AdvectArgs &a, hipStream_t s);
hipError_t launch_reset_counter(int *counter, hipStream_t s);
hipError_t launch_advect_batched(int dim, const BatchArgs &a, int grid_blocks, hipStream_t s);
int batched_blocks_per_cu(int dim);
hipError_t launch_advect_points(int dim, const AdvectArgs &a, hipStream_t s);
hipError_t launch_cg(const CgArgs &a, bool fused, hipStream_t s);
hipError_t launch_ftle(int dim, const FtleArgs &a, hipStream_t s);

}  // namespace lcs
