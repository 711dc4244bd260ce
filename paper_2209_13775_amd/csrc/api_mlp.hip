// api_mlp.hip -- C ABI of the Fourier-feature MLP surrogate: forward,
// backward, loss gradient, Adam and the BF16 weight copies.  Arguments are
// validated before anything is launched; all buffers belong to the caller.

#include <math.h>
#include <string.h>

#include "lcs_internal.h"

namespace {

constexpr long long kChunk = 2048;   // rows per partial sum of a weight gradient
constexpr long long kBChunk = 128;   // rows per partial sum of a bias / head gradient

long long nchunks(long long B) { return (B + kChunk - 1) / kChunk; }
long long nbchunks(long long B) { return (B + kBChunk - 1) / kBChunk; }

// training workspace (BF16): H0 [B][128], then (Z_l, H_l) [B][256] for l = 1..4
// inference workspace (BF16): H0 [B][128], Ha [B][256], Hb [B][256]
long long ws_bytes(long long B, bool training)
{
    const long long per = training ? (long long)lcs::kMlpFeat + 2LL * lcs::kMlpHidden * lcs::kMlpWidth
                                   : (long long)lcs::kMlpFeat + 2LL * lcs::kMlpWidth;
    return 2LL * B * per;
}

long long scratch_bytes(long long B)
{
    const long long nc = nchunks(B), nb = nbchunks(B);
    const long long part = (long long)lcs::kMlpWidth * lcs::kMlpWidth;
    return 2LL * 2 * B * lcs::kMlpWidth + 4LL * (nc * part + nb * (lcs::kMlpWidth + lcs::kHeadPart) + 64);
}

lcs_status check_mlp(const lcs_mlp_t *m)
{
    if (!m) return lcs::set_error(LCS_E_ARG, "mlp descriptor is NULL");
    if (!m->freq || !m->params || !m->params_bf16)
        return lcs::set_error(LCS_E_ARG, "mlp freq, params and params_bf16 must not be NULL");
    if (m->reserved != 0) return lcs::set_error(LCS_E_ARG, "mlp reserved field must be 0");
    for (int a = 0; a < 4; ++a)
        if (!isfinite(m->in_shift[a]) || !isfinite(m->in_scale[a]))
            return lcs::set_error(LCS_E_ARG, "mlp input normalisation must be finite");
    if (!isfinite(m->out_scale)) return lcs::set_error(LCS_E_ARG, "mlp out_scale must be finite");
    return LCS_OK;
}

lcs::MlpDev make_dev(const lcs_mlp_t *m)
{
    lcs::MlpDev d;
    memset(&d, 0, sizeof(d));
    d.freq = m->freq;
    for (int a = 0; a < 4; ++a) {
        d.in_shift[a] = m->in_shift[a];
        d.in_scale[a] = m->in_scale[a];
    }
    d.out_scale = m->out_scale;
    d.params = m->params;
    d.wbf = m->params_bf16;
    return d;
}

struct Ws {
    uint16_t *H0;
    uint16_t *Z[lcs::kMlpHidden + 1];
    uint16_t *H[lcs::kMlpHidden + 1];
};

Ws carve(void *ws, long long B, bool training)
{
    Ws w;
    memset(&w, 0, sizeof(w));
    uint16_t *p = static_cast<uint16_t *>(ws);
    w.H0 = p;
    p += B * lcs::kMlpFeat;
    w.H[0] = w.H0;
    for (int l = 1; l <= lcs::kMlpHidden; ++l) {
        if (training) {
            w.Z[l] = p;
            p += B * lcs::kMlpWidth;
            w.H[l] = p;
            p += B * lcs::kMlpWidth;
        } else {
            // ping-pong between two buffers
            w.H[l] = static_cast<uint16_t *>(ws) + B * lcs::kMlpFeat + ((l - 1) % 2) * B * lcs::kMlpWidth;
        }
    }
    return w;
}

long long check_tiles(const lcs_seed_grid_t *g, int *ct)
{
    long long n = 1;
    for (int a = 0; a < 3; ++a) {
        ct[a] = (int)((g->n[a] + lcs::kCheckTile[a] - 1) / lcs::kCheckTile[a]);
        n *= ct[a];
    }
    return n;
}

lcs_status check_window(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, double t0, double T,
                        double dt, int *nsteps)
{
    lcs_status st;
    if ((st = lcs::validate_velocity(vel)) != LCS_OK) return st;
    if (vel->dim != 3) return lcs::set_error(LCS_E_UNSUPPORTED, "the surrogate path is 3D only");
    if ((st = lcs::validate_seeds(seeds, 3)) != LCS_OK) return st;
    if ((st = lcs::validate_steps(T, dt, nsteps)) != LCS_OK) return st;
    const double t_last = vel->t_first + (double)(vel->n_frames - 1) * vel->dt_frame;
    if (!(isfinite(t0) && t0 >= vel->t_first && t0 <= t_last && t0 + T >= vel->t_first &&
          t0 + T <= t_last))
        return lcs::set_error(LCS_E_TIME_RANGE, "[%g, %g] leaves the frame span", t0, t0 + T);
    return lcs::validate_seed_domain(vel, seeds);
}

}  // namespace

extern "C" {

lcs_status lcs_sub(const float *a, const float *b, int64_t n, float *out, void *stream)
{
    if (!a || !b || !out) return lcs::set_error(LCS_E_ARG, "NULL buffer");
    if (n < 1) return lcs::set_error(LCS_E_SHAPE, "n must be positive");
    hipError_t e = lcs::launch_sub(a, b, n, out, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "sub launch");
    return lcs::clear_error();
}

int64_t lcs_check_tile_count(const lcs_seed_grid_t *seeds)
{
    if (!seeds) return 0;
    int ct[3];
    return check_tiles(seeds, ct);
}

lcs_status lcs_surrogate_compose(const lcs_mlp_t *mlp, const lcs_seed_grid_t *seeds, double t0,
                                 double tau, int32_t n_windows, float *xf, void *stream)
{
    lcs_status st;
    if ((st = check_mlp(mlp)) != LCS_OK) return st;
    if ((st = lcs::validate_seeds(seeds, 3)) != LCS_OK) return st;
    if (!xf) return lcs::set_error(LCS_E_ARG, "xf must not be NULL");
    if (n_windows < 1 || !isfinite(tau) || tau == 0.0 || !isfinite(t0))
        return lcs::set_error(LCS_E_ARG, "need n_windows >= 1 and finite non-zero tau");
    lcs::ComposeArgs A;
    memset(&A, 0, sizeof(A));
    A.P = make_dev(mlp);
    A.g = lcs::seed_tiling(seeds);
    A.ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    A.t0 = t0;
    A.tau = tau;
    A.n_windows = n_windows;
    A.xf = xf;
    hipError_t e = lcs::launch_compose_fused(A, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "surrogate compose launch");
    return lcs::clear_error();
}

lcs_status lcs_surrogate_check(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, double t0,
                               double T, double dt, const float *xf, float tol, float *tile_err,
                               uint8_t *tile_fail, int32_t *n_fail, void *stream)
{
    int nsteps = 0;
    lcs_status st = check_window(vel, seeds, t0, T, dt, &nsteps);
    if (st != LCS_OK) return st;
    if (!xf || !tile_err || !tile_fail || !n_fail)
        return lcs::set_error(LCS_E_ARG, "xf, tile_err, tile_fail and n_fail must not be NULL");
    if (!(tol >= 0.0f)) return lcs::set_error(LCS_E_ARG, "tol must be >= 0");
    lcs::CheckArgs A;
    memset(&A, 0, sizeof(A));
    A.v = lcs::velocity_dev(vel);
    A.g = lcs::seed_tiling(seeds);
    A.t0 = t0;
    A.dt = dt;
    A.nsteps = nsteps;
    A.ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    A.xf = xf;
    A.tile_err = tile_err;
    A.n_tiles = check_tiles(seeds, A.ct);
    hipError_t e = lcs::launch_surrogate_check(A, tol, tile_fail, n_fail, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "surrogate check launch");
    return lcs::clear_error();
}

lcs_status lcs_advect_tiles(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, double t0, double T,
                            double dt, const uint8_t *tile_fail, float *xf, int64_t *cell,
                            uint8_t *flags, void *stream)
{
    int nsteps = 0;
    lcs_status st = check_window(vel, seeds, t0, T, dt, &nsteps);
    if (st != LCS_OK) return st;
    if (!tile_fail || !xf) return lcs::set_error(LCS_E_ARG, "tile_fail and xf must not be NULL");
    lcs::AdvectArgs A;
    memset(&A, 0, sizeof(A));
    A.v = lcs::velocity_dev(vel);
    A.g = lcs::seed_tiling(seeds);
    A.t0 = t0;
    A.dt = dt;
    A.nsteps = nsteps;
    A.ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    A.xf = xf;
    A.cell = reinterpret_cast<long long *>(cell);
    A.flags = flags;
    int ct[3];
    const long long nt = check_tiles(seeds, ct);
    if (nt * 8 > 2147483647LL) return lcs::set_error(LCS_E_SHAPE, "too many tiles");
    hipError_t e = lcs::launch_advect_tiles(A, tile_fail, ct[0], ct[1], nt, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "advect_tiles launch");
    return lcs::clear_error();
}


}  // extern "C"

namespace {

// Workspace of lcs_surrogate_flowmap: per-tile errors and failure marks, the
// failure counter, then (if the whole-grid fallback may be taken) the
// re-bundling workspace of lcs_advect_sorted; each part 256-byte aligned.
struct FlowmapWs {
    float *tile_err;
    uint8_t *tile_fail;
    int *n_fail;
    void *sorted;
    long long sorted_bytes;
    long long bytes;
};

long long align256(long long b) { return (b + 255) / 256 * 256; }

FlowmapWs flowmap_layout(const lcs_velocity_t *vel, const lcs_seed_grid_t *seeds, bool whole,
                         void *base)
{
    int ct[3];
    const long long nt = check_tiles(seeds, ct);
    FlowmapWs w;
    memset(&w, 0, sizeof(w));
    char *p = static_cast<char *>(base);
    long long off = 0;
    w.tile_err = reinterpret_cast<float *>(p + off);
    off += align256(4 * nt);
    w.tile_fail = reinterpret_cast<uint8_t *>(p + off);
    off += align256(nt);
    w.n_fail = reinterpret_cast<int *>(p + off);
    off += 256;
    w.sorted = p + off;
    w.sorted_bytes = whole ? lcs_advect_sorted_workspace_bytes(vel, seeds) : 0;
    off += align256(w.sorted_bytes);
    w.bytes = off;
    return w;
}

}  // namespace

extern "C" {

int64_t lcs_surrogate_flowmap_workspace_bytes(const lcs_velocity_t *vel,
                                              const lcs_seed_grid_t *seeds,
                                              double whole_grid_fraction)
{
    if (!vel || !seeds || lcs::validate_velocity(vel) != LCS_OK ||
        lcs::validate_seeds(seeds, 3) != LCS_OK)
        return 0;
    return flowmap_layout(vel, seeds, whole_grid_fraction < 1.0, nullptr).bytes;
}

lcs_status lcs_surrogate_flowmap(const lcs_mlp_t *mlp, const lcs_velocity_t *vel,
                                 const lcs_seed_grid_t *seeds, double t0, double tau,
                                 int32_t n_windows, double tol, double dt,
                                 double whole_grid_fraction, float *xf, uint8_t *flags,
                                 float *tile_err, int32_t *n_fallback_tiles, int32_t *whole_grid,
                                 void *workspace, int64_t workspace_bytes, void *stream)
{
    lcs_status st;
    if ((st = check_mlp(mlp)) != LCS_OK) return st;
    if (n_windows < 1 || !isfinite(tau) || tau == 0.0)
        return lcs::set_error(LCS_E_ARG, "need n_windows >= 1 and finite non-zero tau");
    const double T = (double)n_windows * tau;
    int nsteps = 0;
    if ((st = check_window(vel, seeds, t0, T, dt, &nsteps)) != LCS_OK) return st;
    if (!xf || !workspace) return lcs::set_error(LCS_E_ARG, "xf and workspace must not be NULL");
    if (!(tol >= 0.0)) return lcs::set_error(LCS_E_ARG, "tol must be >= 0 (inf accepts every tile)");
    if (!(whole_grid_fraction >= 0.0)) return lcs::set_error(LCS_E_ARG, "whole_grid_fraction must be >= 0");
    const bool whole_ok = whole_grid_fraction < 1.0;
    const FlowmapWs w = flowmap_layout(vel, seeds, whole_ok, workspace);
    if (workspace_bytes < w.bytes)
        return lcs::set_error(LCS_E_SHAPE, "workspace of %lld bytes is smaller than the %lld needed",
                              (long long)workspace_bytes, w.bytes);
    hipStream_t s = (hipStream_t)stream;
    const long long ns = seeds->n[0] * seeds->n[1] * seeds->n[2];
    int ct[3];
    const long long nt = check_tiles(seeds, ct);

    // 1. composition of the windows
    lcs::ComposeArgs A;
    memset(&A, 0, sizeof(A));
    A.P = make_dev(mlp);
    A.g = lcs::seed_tiling(seeds);
    A.ns = ns;
    A.t0 = t0;
    A.tau = tau;
    A.n_windows = n_windows;
    A.xf = xf;
    hipError_t e = lcs::launch_compose_fused(A, s);
    if (e != hipSuccess) return lcs::hip_error(e, "surrogate compose launch");
    // 2. check samples against plain RK4 over the whole interval
    lcs::CheckArgs K;
    memset(&K, 0, sizeof(K));
    K.v = lcs::velocity_dev(vel);
    K.g = A.g;
    K.t0 = t0;
    K.dt = dt;
    K.nsteps = nsteps;
    K.ns = ns;
    K.xf = xf;
    K.tile_err = tile_err ? tile_err : w.tile_err;
    K.n_tiles = check_tiles(seeds, K.ct);
    e = lcs::launch_surrogate_check(K, (float)fmin(tol, (double)INFINITY), w.tile_fail, w.n_fail, s);
    if (e == hipSuccess && flags) e = lcs::launch_fill_u8(flags, ns, 0, s);
    if (e != hipSuccess) return lcs::hip_error(e, "surrogate check launch");
    // 3. the number of failing tiles decides the fallback (one synchronisation)
    int nf = 0;
    e = hipMemcpyAsync(&nf, w.n_fail, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return lcs::hip_error(e, "reading the failing-tile count");
    const bool whole = whole_ok && nf > 0 && (double)nf > whole_grid_fraction * (double)nt;
    if (n_fallback_tiles) *n_fallback_tiles = nf;
    if (whole_grid) *whole_grid = whole ? 1 : 0;
    if (whole) {
        // re-bundled RK4 of every seed: the same per-tracer arithmetic as the
        // tile fallback, faster when most tiles fail
        return lcs_advect_sorted(vel, seeds, t0, T, dt, 0, xf, nullptr, flags, w.sorted,
                                 w.sorted_bytes, stream);
    }
    if (nf > 0) {
        lcs::AdvectArgs R;
        memset(&R, 0, sizeof(R));
        R.v = K.v;
        R.g = A.g;
        R.t0 = t0;
        R.dt = dt;
        R.nsteps = nsteps;
        R.ns = ns;
        R.xf = xf;
        R.flags = flags;
        if (nt * 8 > 2147483647LL) return lcs::set_error(LCS_E_SHAPE, "too many tiles");
        e = lcs::launch_advect_tiles(R, w.tile_fail, ct[0], ct[1], nt, s);
        if (e != hipSuccess) return lcs::hip_error(e, "advect_tiles launch");
    }
    return lcs::clear_error();
}

int64_t lcs_mlp_workspace_bytes(int64_t batch, int32_t training)
{
    return batch > 0 ? ws_bytes(batch, training != 0) : 0;
}

int64_t lcs_mlp_backward_scratch_bytes(int64_t batch) { return batch > 0 ? scratch_bytes(batch) : 0; }

lcs_status lcs_mlp_refresh_bf16(const float *params, uint16_t *params_bf16, void *stream)
{
    if (!params || !params_bf16) return lcs::set_error(LCS_E_ARG, "params and params_bf16 must not be NULL");
    hipError_t e = lcs::launch_refresh_bf16(params, params_bf16, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "refresh_bf16 launch");
    return lcs::clear_error();
}

lcs_status lcs_mlp_forward(const lcs_mlp_t *mlp, const float *xt, int64_t batch, float *dx,
                           void *workspace, int64_t workspace_bytes, int32_t training, void *stream)
{
    lcs_status st;
    if ((st = check_mlp(mlp)) != LCS_OK) return st;
    if (!xt || !dx || !workspace) return lcs::set_error(LCS_E_ARG, "xt, dx and workspace must not be NULL");
    if (batch < 1 || batch > (1LL << 31) - 1) return lcs::set_error(LCS_E_SHAPE, "batch out of range");
    if (workspace_bytes < ws_bytes(batch, training != 0))
        return lcs::set_error(LCS_E_SHAPE, "workspace of %lld bytes is smaller than the %lld needed",
                              (long long)workspace_bytes, ws_bytes(batch, training != 0));
    hipStream_t s = (hipStream_t)stream;
    const lcs::MlpDev P = make_dev(mlp);
    const Ws w = carve(workspace, batch, training != 0);
    hipError_t e = lcs::launch_features(P, xt, batch, w.H0, s);
    for (int l = 0; l < lcs::kMlpHidden && e == hipSuccess; ++l) {
        lcs::GemmArgs g;
        memset(&g, 0, sizeof(g));
        g.A = w.H[l];
        g.Bt = P.wbf + lcs::mlp_off_bf16(l) + (long long)lcs::mlp_in_width(l) * lcs::kMlpWidth;
        g.bt_frag = 1;                                    // W_l^T, fragment order
        g.M = batch;
        g.N = lcs::kMlpWidth;
        g.K = lcs::mlp_in_width(l);
        g.bias = P.params + lcs::mlp_off_b(l);
        g.H = w.H[l + 1];
        g.Z = training ? w.Z[l + 1] : nullptr;
        e = lcs::launch_gemm(g, false, s);
    }
    if (e == hipSuccess) e = lcs::launch_head_fwd(P, w.H[lcs::kMlpHidden], batch, dx, s);
    if (e != hipSuccess) return lcs::hip_error(e, "mlp forward launch");
    return lcs::clear_error();
}

lcs_status lcs_mlp_backward(const lcs_mlp_t *mlp, const void *workspace, const float *ddx,
                            int64_t batch, float *grads, void *scratch, int64_t scratch_size,
                            void *stream)
{
    lcs_status st;
    if ((st = check_mlp(mlp)) != LCS_OK) return st;
    if (!workspace || !ddx || !grads || !scratch)
        return lcs::set_error(LCS_E_ARG, "workspace, ddx, grads and scratch must not be NULL");
    if (batch < 1 || batch > (1LL << 31) - 1) return lcs::set_error(LCS_E_SHAPE, "batch out of range");
    if (scratch_size < scratch_bytes(batch))
        return lcs::set_error(LCS_E_SHAPE, "scratch of %lld bytes is smaller than the %lld needed",
                              (long long)scratch_size, scratch_bytes(batch));
    hipStream_t s = (hipStream_t)stream;
    const lcs::MlpDev P = make_dev(mlp);
    const Ws w = carve(const_cast<void *>(workspace), batch, true);
    const long long nc = nchunks(batch), nb = nbchunks(batch);
    uint16_t *dA = static_cast<uint16_t *>(scratch);
    uint16_t *dB = dA + batch * lcs::kMlpWidth;
    float *part = reinterpret_cast<float *>(dB + batch * lcs::kMlpWidth);
    float *part_b = part + nc * (long long)lcs::kMlpWidth * lcs::kMlpWidth;
    float *part_h = part_b + nb * lcs::kMlpWidth;

    hipError_t e = lcs::launch_head_bwd(P, ddx, w.Z[lcs::kMlpHidden], w.H[lcs::kMlpHidden], batch, dA,
                                        kBChunk, (int)nb, part_h, s);
    if (e == hipSuccess)
        e = lcs::launch_reduce_chunks(part_h, (int)nb, lcs::kHeadPart, grads + lcs::kOffWh, s);
    uint16_t *cur = dA, *nxt = dB;
    for (int l = lcs::kMlpHidden - 1; l >= 0 && e == hipSuccess; --l) {
        const int K = lcs::mlp_in_width(l);
        lcs::WgradArgs wg;
        wg.X = w.H[l];
        wg.D = cur;
        wg.M = batch;
        wg.K = K;
        wg.N = lcs::kMlpWidth;
        wg.chunk = kChunk;
        wg.part = part;
        e = lcs::launch_wgrad(wg, (int)nc, s);
        if (e == hipSuccess)
            e = lcs::launch_reduce_chunks(part, (int)nc, (long long)K * lcs::kMlpWidth,
                                          grads + lcs::mlp_off_w(l), s);
        if (e == hipSuccess) e = lcs::launch_colsum(cur, batch, lcs::kMlpWidth, kBChunk, (int)nb, part_b, s);
        if (e == hipSuccess)
            e = lcs::launch_reduce_chunks(part_b, (int)nb, lcs::kMlpWidth, grads + lcs::mlp_off_b(l), s);
        if (l > 0 && e == hipSuccess) {
            lcs::GemmArgs g;
            memset(&g, 0, sizeof(g));
            g.A = cur;                                        // dZ_{l+1} [B][256]
            g.Bt = P.wbf + lcs::mlp_off_bf16(l);              // W_l as [in][out] = Bt[N=in][K=out]
            g.bt_frag = 1;                                    // fragment order
            g.M = batch;
            g.N = K;
            g.K = lcs::kMlpWidth;
            g.H = nxt;                                        // dZ_l
            g.Z = w.Z[l];
            e = lcs::launch_gemm(g, true, s);
            uint16_t *t = cur;
            cur = nxt;
            nxt = t;
        }
    }
    if (e != hipSuccess) return lcs::hip_error(e, "mlp backward launch");
    return lcs::clear_error();
}

lcs_status lcs_mse_grad(const float *pred, const float *target, int64_t n, float *grad, double *loss,
                        void *stream)
{
    if (!pred || !target) return lcs::set_error(LCS_E_ARG, "pred and target must not be NULL");
    if (!grad && !loss) return lcs::set_error(LCS_E_ARG, "grad and loss are both NULL");
    if (n < 1) return lcs::set_error(LCS_E_SHAPE, "n must be positive");
    hipError_t e = lcs::launch_mse(pred, target, n, (float)(2.0 / (double)n), grad, loss,
                                   1.0 / (double)n, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "mse launch");
    return lcs::clear_error();
}

lcs_status lcs_adam_step(float *params, const float *grads, float *m, float *v, int64_t n, float lr,
                         float beta1, float beta2, float eps, int32_t step, void *stream)
{
    if (!params || !grads || !m || !v) return lcs::set_error(LCS_E_ARG, "NULL buffer");
    if (n < 1) return lcs::set_error(LCS_E_SHAPE, "n must be positive");
    if (step < 1) return lcs::set_error(LCS_E_ARG, "step counts from 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && isfinite(lr)))
        return lcs::set_error(LCS_E_ARG, "bad Adam hyper-parameters");
    lcs::AdamArgs a;
    a.lr = lr;
    a.beta1 = beta1;
    a.beta2 = beta2;
    a.eps = eps;
    a.c1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)step)));
    a.c2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)step)));
    hipError_t e = lcs::launch_adam(params, grads, m, v, n, a, (hipStream_t)stream);
    if (e != hipSuccess) return lcs::hip_error(e, "adam launch");
    return lcs::clear_error();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Fused training: lcs_mlp_train runs Adam steps on consecutive batches of a
// resident training set, four launches per step (train.hip).
// ---------------------------------------------------------------------------
namespace {

struct TrainWs {
    uint16_t *dgelu[lcs::kMlpHidden], *ht[lcs::kMlpHidden], *dzt[lcs::kMlpHidden];
    float *dy, *part_head, *part_w;
    double *part_loss;
    long long bytes;
};

long long train_tiles(long long B) { return (B + 127) / 128; }

TrainWs train_layout(long long B, void *base)
{
    const long long nt = train_tiles(B), Bp = nt * 128;
    const long long nch = (Bp + lcs::kWgradChunk - 1) / lcs::kWgradChunk;
    TrainWs w;
    memset(&w, 0, sizeof(w));
    char *p = static_cast<char *>(base);
    long long off = 0;
    auto take = [&](long long bytes) {
        char *q = p ? p + off : nullptr;
        off += align256(bytes);
        return q;
    };
    for (int l = 0; l < lcs::kMlpHidden; ++l) {
        w.dgelu[l] = reinterpret_cast<uint16_t *>(take(2 * Bp * lcs::kMlpWidth));
        w.ht[l] = reinterpret_cast<uint16_t *>(take(2 * Bp * lcs::mlp_in_width(l)));
        w.dzt[l] = reinterpret_cast<uint16_t *>(take(2 * Bp * lcs::kMlpWidth));
    }
    w.dy = reinterpret_cast<float *>(take(4 * 3 * Bp));
    w.part_head = reinterpret_cast<float *>(take(4 * nt * lcs::kHeadPart));
    w.part_loss = reinterpret_cast<double *>(take(8 * nt));
    w.part_w = reinterpret_cast<float *>(take(4 * nch * lcs::kMlpParams));
    w.bytes = off;
    return w;
}

}  // namespace

extern "C" {

int64_t lcs_mlp_train_workspace_bytes(int64_t batch)
{
    if (batch < 1 || batch > (1LL << 31) - 1) return 0;
    return train_layout(batch, nullptr).bytes;
}

lcs_status lcs_mlp_train(const lcs_mlp_t *mlp, float *params, uint16_t *params_bf16, const float *xt,
                         const float *target, int64_t n, int64_t batch, int32_t first_step,
                         int32_t n_steps, int32_t total_steps, float lr, float lr_final, float beta1,
                         float beta2, float eps, float *m, float *v, double *losses, float *grads,
                         void *workspace, int64_t workspace_bytes, void *stream)
{
    lcs_status st;
    if ((st = check_mlp(mlp)) != LCS_OK) return st;
    if (!params || params != mlp->params || !params_bf16 || params_bf16 != mlp->params_bf16)
        return lcs::set_error(LCS_E_ARG, "params and params_bf16 must be the descriptor's buffers");
    if (!xt || !target || !m || !v || !workspace)
        return lcs::set_error(LCS_E_ARG, "xt, target, m, v and workspace must not be NULL");
    if (batch < 1 || batch > (1LL << 31) - 1 || n < batch)
        return lcs::set_error(LCS_E_SHAPE, "need 1 <= batch <= n and batch < 2^31");
    if (first_step < 1 || n_steps < 0 || total_steps < 1)
        return lcs::set_error(LCS_E_ARG, "steps count from 1; n_steps >= 0; total_steps >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f &&
          isfinite(lr) && isfinite(lr_final)))
        return lcs::set_error(LCS_E_ARG, "bad Adam hyper-parameters");
    const TrainWs need = train_layout(batch, nullptr);
    if (workspace_bytes < need.bytes)
        return lcs::set_error(LCS_E_SHAPE, "workspace of %lld bytes is smaller than the %lld needed",
                              (long long)workspace_bytes, need.bytes);
    const TrainWs w = train_layout(batch, workspace);
    hipStream_t s = (hipStream_t)stream;
    lcs::TrainArgs A;
    memset(&A, 0, sizeof(A));
    A.P = make_dev(mlp);
    A.ld = n;
    A.B = batch;
    A.n_tiles = train_tiles(batch);
    A.Bp = A.n_tiles * 128;
    A.n_chunks = (A.Bp + lcs::kWgradChunk - 1) / lcs::kWgradChunk;
    A.mse_scale = (float)(2.0 / (3.0 * (double)batch));
    A.loss_mult = 1.0 / (3.0 * (double)batch);
    for (int l = 0; l < lcs::kMlpHidden; ++l) {
        A.dgelu[l] = w.dgelu[l];
        A.ht[l] = w.ht[l];
        A.dzt[l] = w.dzt[l];
    }
    A.dy = w.dy;
    A.part_head = w.part_head;
    A.part_loss = w.part_loss;
    A.part_w = w.part_w;
    A.params = params;
    A.wbf = params_bf16;
    A.m = m;
    A.v = v;
    const long long nb = n / batch;
    hipError_t e = hipSuccess;
    for (int k = 0; k < n_steps && e == hipSuccess; ++k) {
        const long long step = (long long)first_step + k;
        const long long b = (step - 1) % nb;
        A.xt = xt + b * batch;
        A.target = target + b * batch;
        A.loss = losses ? losses + k : nullptr;
        A.grads = (k + 1 == n_steps) ? grads : nullptr;
        // cosine decay from lr (step 1) to lr_final (step total_steps)
        const double frac = (double)(step - 1) / (double)(total_steps > 1 ? total_steps - 1 : 1);
        lcs::AdamArgs ad;
        ad.lr = (float)(lr_final + 0.5 * ((double)lr - lr_final) * (1.0 + cos(M_PI * fmin(frac, 1.0))));
        ad.beta1 = beta1;
        ad.beta2 = beta2;
        ad.eps = eps;
        ad.c1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)step)));
        ad.c2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)step)));
        e = lcs::launch_train_step(A, ad, s);
    }
    if (e != hipSuccess) return lcs::hip_error(e, "mlp train launch");
    return lcs::clear_error();
}

}  // extern "C"
