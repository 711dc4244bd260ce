"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/lcs.h declares, and rejects bad arguments with the
documented status codes before anything is launched."""
import ctypes as C

import pytest

from paper_2209_13775_amd import lcs


def test_exports_every_declared_symbol():
    names = lcs.declared_entry_points()
    assert "lcs_advect" in names and "lcs_cg_tensor" in names and "lcs_ftle" in names
    L = C.CDLL(lcs.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def _vel(dim=2, n=(5, 4, 1), frames=3, t_first=0.0, dt_frame=1.0, periodic=0):
    v = lcs.lcs_velocity_t()
    v.dim = dim
    v.n_frames = frames
    for a in range(3):
        v.n[a] = n[a]
        v.origin[a] = 0.0
        v.spacing[a] = 0.25
    v.periodic_mask = periodic
    v.t_first = t_first
    v.dt_frame = dt_frame
    for c in range(3):
        v.u[c] = 0x1000 if c < dim else None   # never dereferenced: validation fails first
    return v


def _seeds(dim=2, n=(3, 3, 1), origin=(0.1, 0.1, 0.0), spacing=(0.2, 0.2, 1.0), periodic=0):
    s = lcs.lcs_seed_grid_t()
    s.dim = dim
    s.periodic_mask = periodic
    for a in range(3):
        s.n[a] = n[a]
        s.origin[a] = origin[a]
        s.spacing[a] = spacing[a]
    return s


def _advect(v, s, t0, T, dt, xf=0x2000):
    return lcs.lib().lcs_advect(C.byref(v) if v is not None else None,
                                C.byref(s) if s is not None else None,
                                t0, T, dt, xf, None, None, None)


@pytest.mark.parametrize("case,expect", [
    ("null_vel", lcs.LCS_E_ARG),
    ("null_seeds", lcs.LCS_E_ARG),
    ("null_xf", lcs.LCS_E_ARG),
    ("bad_dim", lcs.LCS_E_ARG),
    ("one_frame", lcs.LCS_E_SHAPE),
    ("one_node", lcs.LCS_E_SHAPE),
    ("nonint_steps", lcs.LCS_E_STEP),
    ("sign_mismatch", lcs.LCS_E_STEP),
    ("zero_T", lcs.LCS_E_STEP),
    ("time_range", lcs.LCS_E_TIME_RANGE),
    ("seed_outside", lcs.LCS_E_SEED_DOMAIN),
    ("periodic_seed_on_closed_axis", lcs.LCS_E_ARG),
    ("periodic_seed_partial_period", lcs.LCS_E_ARG),
    ("periodic_seed_full_period_passes", lcs.LCS_E_TIME_RANGE),
    ("bad_layout", lcs.LCS_E_ARG),
    ("xyzw_in_2d", lcs.LCS_E_ARG),
    ("misaligned_interleaved", lcs.LCS_E_ARG),
    ("frame_over_4gib", lcs.LCS_E_SHAPE),
    ("misaligned_tpair_2d", lcs.LCS_E_ARG),
    ("misaligned_tpair", lcs.LCS_E_ARG),
    ("empty_seed_axis", lcs.LCS_E_SHAPE),
    ("single_seed_axis", lcs.LCS_E_SHAPE),
    ("seed_grid_over_2g", lcs.LCS_E_SHAPE),
    ("seed_dim_mismatch", lcs.LCS_E_ARG),
])
def test_advect_validation(case, expect):
    v, s = _vel(), _seeds()
    t0, T, dt, xf = 0.0, 1.0, 0.1, 0x2000
    if case == "null_vel":
        v = None
    elif case == "null_seeds":
        s = None
    elif case == "null_xf":
        xf = None
    elif case == "bad_dim":
        v.dim = 4
    elif case == "one_frame":
        v.n_frames = 1
    elif case == "one_node":
        v.n[1] = 1
    elif case == "nonint_steps":
        dt = 0.3
    elif case == "sign_mismatch":
        dt = -0.1
    elif case == "zero_T":
        T = 0.0
    elif case == "time_range":
        T = 2.5            # frames span [0, 2]
    elif case == "seed_outside":
        s.origin[0] = 0.7  # 0.7 + 2*0.2 = 1.1 > 4*0.25
    elif case == "periodic_seed_on_closed_axis":
        s.periodic_mask = 1
    elif case in ("periodic_seed_partial_period", "periodic_seed_full_period_passes"):
        # velocity period 5 x 0.25 = 1.25; seeds 3 x 0.2 = 0.6 cover part of it
        v.periodic_mask = s.periodic_mask = 1
        if case.endswith("passes"):
            s.spacing[0] = 1.25 / 3        # full period: validation goes on to the
            T = 2.5                        # time range, which fails instead
    elif case == "bad_layout":
        v.layout = 7
    elif case == "xyzw_in_2d":
        v.layout = lcs.LCS_LAYOUT_XYZW
    elif case == "misaligned_interleaved":
        v.layout = lcs.LCS_LAYOUT_XYZ
        v.u[0] = 0x1004                # 2D interleaved frames need 8-byte alignment
    elif case == "misaligned_tpair_2d":
        v.layout = lcs.LCS_LAYOUT_TPAIR
        v.u[0] = 0x1008                # 2D time-paired records need 16-byte alignment too
    elif case == "misaligned_tpair":
        v.dim, v.n[2] = 3, 4
        v.layout = lcs.LCS_LAYOUT_TPAIR
        v.u[0] = 0x1008                # time-paired records need 16-byte alignment
        s.dim, s.n[2], s.spacing[2] = 3, 1, 0.2
    elif case == "empty_seed_axis":
        s.n[0] = 0                     # no seeds: the gradient needs two per axis
    elif case == "single_seed_axis":
        s.n[1] = 1
    elif case == "seed_grid_over_2g":
        s.n[0], s.n[1] = 1 << 16, 1 << 15     # 2^31 seeds
        s.spacing[0] = s.spacing[1] = 1e-6
    elif case == "seed_dim_mismatch":
        s.dim = 3
    elif case == "frame_over_4gib":
        v.layout = lcs.LCS_LAYOUT_XYZ  # 2^29 nodes x 8 B per interleaved 2D frame = 4 GiB
        v.n[0], v.n[1] = 1 << 15, (1 << 14) + 1
    st = _advect(v, s, t0, T, dt, xf)
    assert st == expect, lcs.lcs_last_error()
    assert lcs.lcs_last_error() != ""


def test_frame_size_limit_accepts_4gib():
    """A frame array of exactly 4 GiB passes validation (32-bit byte offsets
    reach every record); the call then fails on its time range instead."""
    v, s = _vel(), _seeds()
    v.n[0], v.n[1] = 1 << 15, 1 << 15        # 2^30 nodes x 4 B per component
    st = _advect(v, s, 0.0, 2.5, 0.1)
    assert st == lcs.LCS_E_TIME_RANGE, lcs.lcs_last_error()


def test_other_entry_points_validate():
    L = lcs.lib()
    s = _seeds()
    assert L.lcs_cg_tensor(C.byref(s), None, None, 0x10, None, None) == lcs.LCS_E_ARG
    assert L.lcs_cg_tensor(C.byref(s), 0x10, None, None, None, None) == lcs.LCS_E_ARG
    assert L.lcs_ftle(4, 10, 0x10, 1.0, 0x20, None, None) == lcs.LCS_E_ARG
    assert L.lcs_ftle(3, 0, 0x10, 1.0, 0x20, None, None) == lcs.LCS_E_SHAPE
    assert L.lcs_ftle(3, 10, 0x10, 0.0, 0x20, None, None) == lcs.LCS_E_ARG
    assert L.lcs_ftle(3, 10, 0x10, 1.0, None, None, None) == lcs.LCS_E_ARG
    assert L.lcs_cg_ftle(C.byref(s), 0x10, None, 1.0, None, None, None, None) == lcs.LCS_E_ARG
    v = _vel()
    assert L.lcs_advect_points(C.byref(v), 0x10, 0x20, 0, 1.0, 0.1, 0x30, None, None, None) == \
        lcs.LCS_E_SHAPE
    assert L.lcs_advect_points(C.byref(v), None, 0x20, 5, 1.0, 0.1, 0x30, None, None, None) == \
        lcs.LCS_E_ARG
    assert lcs.lcs_version() >= 100


def test_batched_validation():
    L = lcs.lib()
    v, s = _vel(), _seeds()
    win = (lcs.lcs_window_t * 2)(lcs.lcs_window_t(0.0, 1.0), lcs.lcs_window_t(0.5, 1.0))
    fake_plan = C.c_void_p(0x1)      # never dereferenced: validation fails first
    assert L.lcs_advect_batched(None, C.byref(v), C.byref(s), win, 2, 0.1, 0x10, None, None,
                                None) == lcs.LCS_E_ARG
    assert L.lcs_advect_batched(fake_plan, C.byref(v), C.byref(s), win, 0, 0.1, 0x10, None, None,
                                None) == lcs.LCS_E_SHAPE
    assert L.lcs_advect_batched(fake_plan, C.byref(v), C.byref(s), win, 193, 0.1, 0x10, None,
                                None, None) == lcs.LCS_E_SHAPE
    bad = (lcs.lcs_window_t * 2)(lcs.lcs_window_t(0.0, 1.0), lcs.lcs_window_t(1.5, 1.0))
    assert L.lcs_advect_batched(fake_plan, C.byref(v), C.byref(s), bad, 2, 0.1, 0x10, None, None,
                                None) == lcs.LCS_E_TIME_RANGE
    bad2 = (lcs.lcs_window_t * 2)(lcs.lcs_window_t(0.0, 1.0), lcs.lcs_window_t(0.5, 0.35))
    assert L.lcs_advect_batched(fake_plan, C.byref(v), C.byref(s), bad2, 2, 0.1, 0x10, None,
                                None, None) == lcs.LCS_E_STEP
    assert L.lcs_plan_create(None, None) == lcs.LCS_E_ARG
    assert L.lcs_plan_destroy(None) == lcs.LCS_OK


def test_mesh_entry_points_validate():
    """Mesh calls reject bad arguments on the host, before any device work."""
    L = lcs.lib()
    d = lcs.lcs_mesh_desc_t()
    out = C.c_void_p()
    assert L.lcs_mesh_create(None, C.byref(out), None) == lcs.LCS_E_ARG
    assert L.lcs_mesh_create(C.byref(d), None, None) == lcs.LCS_E_ARG
    d.dim, d.n_nodes, d.n_cells, d.nodes, d.cells = 4, 4, 1, 0x10, 0x20
    assert L.lcs_mesh_create(C.byref(d), C.byref(out), None) == lcs.LCS_E_ARG
    d.dim = 3
    d.reserved = 1
    assert L.lcs_mesh_create(C.byref(d), C.byref(out), None) == lcs.LCS_E_ARG
    d.reserved = 0
    d.n_nodes = 0
    assert L.lcs_mesh_create(C.byref(d), C.byref(out), None) == lcs.LCS_E_SHAPE
    d.n_nodes, d.n_cells = 1 << 28, 1
    assert L.lcs_mesh_create(C.byref(d), C.byref(out), None) == lcs.LCS_E_SHAPE
    d.n_nodes, d.n_cells = 4, 1 << 30
    assert L.lcs_mesh_create(C.byref(d), C.byref(out), None) == lcs.LCS_E_SHAPE
    d.n_cells, d.cells = 1, None
    assert L.lcs_mesh_create(C.byref(d), C.byref(out), None) == lcs.LCS_E_ARG
    assert out.value is None
    info = lcs.lcs_mesh_info_t()
    assert L.lcs_mesh_info(None, C.byref(info)) == lcs.LCS_E_ARG
    f = lcs.lcs_mesh_frames_t()
    s = lcs.lcs_seed_grid_t()
    assert L.lcs_mesh_advect(None, C.byref(f), C.byref(s), 0.0, 1.0, 0.1, 0x10, None, None,
                             None) == lcs.LCS_E_ARG
    assert L.lcs_mesh_advect_points(None, C.byref(f), 0x10, 0x20, 4, 1.0, 0.1, 0x30, None, None,
                                    None) == lcs.LCS_E_ARG
    assert L.lcs_mesh_locate(None, 0x10, 4, 0x20, None, None) == lcs.LCS_E_ARG
    assert L.lcs_mesh_velocity_at(None, C.byref(f), 0x10, 0x20, 4, 0x30, None, None) == lcs.LCS_E_ARG
    L.lcs_mesh_destroy(None)


def test_aux_sorted_validates():
    L = lcs.lib()
    v, s = _vel(), _seeds()
    d = (C.c_double * 3)(0.01, 0.01, 0.0)
    bad = (C.c_double * 3)(0.01, 0.0, 0.0)
    args = (0.0, 1.0, 0.1, 0, 0x2000, 0x3000, None, 0x4000, 1 << 20, None)
    assert L.lcs_advect_aux_sorted(C.byref(v), C.byref(s), None, *args) == lcs.LCS_E_ARG
    assert L.lcs_advect_aux_sorted(C.byref(v), C.byref(s), bad, *args) == lcs.LCS_E_ARG
    assert L.lcs_advect_aux_sorted(C.byref(v), C.byref(s), d, 0.0, 1.0, 0.1, 0, 0x2000, None,
                                   None, 0x4000, 1 << 20, None) == lcs.LCS_E_ARG
    assert L.lcs_advect_aux_sorted(C.byref(v), C.byref(s), d, 0.0, 1.0, 0.1, 0, 0x2000, 0x3000,
                                   None, 0x4000, 16, None) == lcs.LCS_E_SHAPE   # workspace too small
    big = _seeds(n=(30, 30, 1), spacing=(0.02, 0.02, 1.0))   # 2*dim auxiliary tracers per seed
    need = L.lcs_advect_aux_sorted_workspace_bytes(C.byref(v), C.byref(big))
    assert need > L.lcs_advect_sorted_workspace_bytes(C.byref(v), C.byref(big)) > 0


def test_frames_interleave_floats():
    v = _vel(dim=3, n=(5, 4, 3), frames=6)
    L = lcs.lib()
    assert L.lcs_frames_interleave_floats(C.byref(v), lcs.LCS_LAYOUT_XYZ, 4) == 4 * 60 * 3
    assert L.lcs_frames_interleave_floats(C.byref(v), lcs.LCS_LAYOUT_XYZW, 4) == 4 * 60 * 4
    assert L.lcs_frames_interleave_floats(C.byref(v), lcs.LCS_LAYOUT_TPAIR, 4) == 3 * 6 * 4 * 3 * 6
    assert L.lcs_frames_interleave_floats(C.byref(v), lcs.LCS_LAYOUT_TPAIR, 1) == -1
    assert L.lcs_frames_interleave_floats(C.byref(v), 9, 4) == -1
    v2 = _vel()                                            # 2D, 5 x 4 nodes
    assert L.lcs_frames_interleave_floats(C.byref(v2), lcs.LCS_LAYOUT_TPAIR, 3) == 2 * 6 * 4 * 4
    assert L.lcs_frames_interleave_floats(C.byref(v2), lcs.LCS_LAYOUT_XYZW, 3) == -1


def test_frames_interleave_validates():
    L = lcs.lib()
    v = _vel()
    out_desc = lcs.lcs_velocity_t()
    assert L.lcs_frames_interleave(C.byref(v), lcs.LCS_LAYOUT_XYZW, 0, 2, 0x1000, C.byref(out_desc),
                                   None) == lcs.LCS_E_ARG          # XYZW is 3D only
    assert L.lcs_frames_interleave(C.byref(v), lcs.LCS_LAYOUT_TPAIR, 0, 2, 0x1008, C.byref(out_desc),
                                   None) == lcs.LCS_E_ARG          # TPAIR output 16-byte aligned
    assert L.lcs_frames_interleave(C.byref(v), lcs.LCS_LAYOUT_XYZ, 0, 1, 0x1000, C.byref(out_desc),
                                   None) == lcs.LCS_E_SHAPE        # fewer than 2 frames
    assert L.lcs_frames_interleave(C.byref(v), lcs.LCS_LAYOUT_XYZ, 1, 9, 0x1000, C.byref(out_desc),
                                   None) == lcs.LCS_E_SHAPE        # past the last frame
    assert L.lcs_frames_interleave(C.byref(v), lcs.LCS_LAYOUT_XYZ, 0, 2, None, C.byref(out_desc),
                                   None) == lcs.LCS_E_ARG
    v.layout = lcs.LCS_LAYOUT_XYZ
    assert L.lcs_frames_interleave(C.byref(v), lcs.LCS_LAYOUT_XYZ, 0, 2, 0x1000, C.byref(out_desc),
                                   None) == lcs.LCS_E_ARG          # source must be SoA


def test_sorted_workspace_follows_the_bin_rule():
    """Sort bins are one cell wide while their Morton keys fit in 24 bits, else
    two cells: a 4097 x 4096 grid (25 bits at one cell, 23 at two) needs the
    same bin histogram as a 2048 x 4096 grid and half that of 4096 x 4096."""
    L = lcs.lib()
    s = _seeds()

    def ws(n):
        v = _vel(n=n)
        return L.lcs_advect_sorted_workspace_bytes(C.byref(v), C.byref(s))

    def hist_bytes(key_bits):   # counts + scan block sums, each rounded up to 256 B
        nk = 1 << key_bits
        return 4 * nk + (4 * (nk // 1024 + 1) + 255) // 256 * 256

    a, b, c = ws((4096, 4096, 1)), ws((4097, 4096, 1)), ws((2048, 4096, 1))
    assert a > 0 and b > 0 and c > 0
    assert b == c
    assert a - c == hist_bytes(24) - hist_bytes(23)


def test_tuned_and_surrogate_flowmap_validate():
    """lcs_advect_tuned and lcs_surrogate_flowmap reject bad arguments before
    any device work (the fake pointers are never dereferenced)."""
    L = lcs.lib()
    v, s = _vel(), _seeds()
    fake_plan = C.c_void_p(0x1)
    c1 = (C.c_int32 * 2)(0, 100)
    cneg = (C.c_int32 * 2)(0, -5)
    args = lambda plan, cand, nc: (plan, C.byref(v), C.byref(s), 0.0, 1.0, 0.1, 0x10, None, None,
                                   None, 0, cand, nc, None, None, None)
    assert L.lcs_advect_tuned(*args(None, c1, 2)) == lcs.LCS_E_ARG
    assert L.lcs_advect_tuned(*args(fake_plan, c1, 0)) == lcs.LCS_E_ARG
    assert L.lcs_advect_tuned(*args(fake_plan, c1, 17)) == lcs.LCS_E_ARG
    assert L.lcs_advect_tuned(*args(fake_plan, cneg, 2)) == lcs.LCS_E_ARG
    v3 = _vel(dim=3, n=(6, 6, 6), periodic=7)
    v3.spacing[0] = v3.spacing[1] = v3.spacing[2] = 1.0
    s3 = _seeds(dim=3, n=(4, 4, 4), origin=(0.0, 0.0, 0.0), spacing=(1.5, 1.5, 1.5), periodic=7)
    m = lcs.lcs_mlp_t()
    m.freq, m.params, m.params_bf16 = 0x100, 0x200, 0x300
    for a in range(4):
        m.in_scale[a] = 1.0
    m.out_scale = 1.0
    ws_need = L.lcs_surrogate_flowmap_workspace_bytes(C.byref(v3), C.byref(s3), 0.25)
    assert ws_need > L.lcs_surrogate_flowmap_workspace_bytes(C.byref(v3), C.byref(s3), 1.0) > 0
    nf, wh = C.c_int32(), C.c_int32()

    def call(mlp=C.byref(m), tol=1e-3, frac=0.25, xf=0x10, ws=0x1000, wsb=None, tau=0.5, nw=2):
        return L.lcs_surrogate_flowmap(mlp, C.byref(v3), C.byref(s3), 0.0, tau, nw, tol, 0.1, frac,
                                       xf, None, None, C.byref(nf), C.byref(wh), ws,
                                       ws_need if wsb is None else wsb, None)
    assert call(mlp=None) == lcs.LCS_E_ARG
    assert call(tol=-1.0) == lcs.LCS_E_ARG
    assert call(tol=float("nan")) == lcs.LCS_E_ARG
    assert call(frac=-0.5) == lcs.LCS_E_ARG
    assert call(xf=None) == lcs.LCS_E_ARG
    assert call(ws=None) == lcs.LCS_E_ARG
    assert call(nw=0) == lcs.LCS_E_ARG
    assert call(wsb=ws_need - 1) == lcs.LCS_E_SHAPE
    assert call(tau=1.5) == lcs.LCS_E_TIME_RANGE       # 2 x 1.5 leaves the frames' [0, 2]
    v2 = _vel()
    assert L.lcs_surrogate_flowmap(C.byref(m), C.byref(v2), C.byref(s), 0.0, 0.5, 2, 1e-3, 0.1,
                                   0.25, 0x10, None, None, None, None, 0x1000, 1 << 20,
                                   None) == lcs.LCS_E_UNSUPPORTED


def test_mlp_train_validates():
    """lcs_mlp_train rejects bad arguments before any device work (the fake
    pointers are never dereferenced); its workspace grows with the batch and
    covers whole 128-sample tiles."""
    L = lcs.lib()
    m = lcs.lcs_mlp_t()
    m.freq, m.params, m.params_bf16 = 0x100, 0x200, 0x300
    for a in range(4):
        m.in_scale[a] = 1.0
    m.out_scale = 1.0
    w1, w128, w129 = (L.lcs_mlp_train_workspace_bytes(b) for b in (1, 128, 129))
    assert 0 < w1 == w128 < w129
    assert L.lcs_mlp_train_workspace_bytes(0) == 0
    need = L.lcs_mlp_train_workspace_bytes(256)

    def call(mlp=C.byref(m), params=0x200, bf=0x300, xt=0x400, n=1024, batch=256, first=1, ns=2,
             total=2, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, mm=0x500, vv=0x600, ws=0x700, wsb=need):
        return L.lcs_mlp_train(mlp, params, bf, xt, 0x800, n, batch, first, ns, total, lr, 1e-4, b1, b2,
                               eps, mm, vv, None, None, ws, wsb, None)
    assert call(mlp=None) == lcs.LCS_E_ARG
    assert call(params=0x204) == lcs.LCS_E_ARG          # not the descriptor's masters
    assert call(bf=None) == lcs.LCS_E_ARG
    assert call(xt=None) == lcs.LCS_E_ARG
    assert call(mm=None) == lcs.LCS_E_ARG
    assert call(ws=None) == lcs.LCS_E_ARG
    assert call(batch=2048) == lcs.LCS_E_SHAPE           # batch > n
    assert call(batch=0) == lcs.LCS_E_SHAPE
    assert call(first=0) == lcs.LCS_E_ARG
    assert call(ns=-1) == lcs.LCS_E_ARG
    assert call(total=0) == lcs.LCS_E_ARG
    assert call(b1=1.0) == lcs.LCS_E_ARG
    assert call(eps=0.0) == lcs.LCS_E_ARG
    assert call(lr=float("nan")) == lcs.LCS_E_ARG
    assert call(wsb=need - 1) == lcs.LCS_E_SHAPE
    assert call(ns=0) == lcs.LCS_OK                       # zero steps: nothing launched
