"""FP64 CPU oracle for the LCS flow-map / FTLE path (test infrastructure).

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product path (the HIP library and its binding)
never imports it and never falls back to it.

The arithmetic lives in ``lcs_oracle.c`` (plain C, FP64, -ffp-contract=off)
and ``mlp_ref.py`` (NumPy FP64); this module only marshals NumPy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lcs_oracle.c")
_LIB = os.path.join(_HERE, "liblcs_oracle.so")

FLAG_OUT = 1
FLAG_NONFINITE = 2
FLAG_STENCIL_OUT = 4
FLAG_TIME_OUT = 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Vel(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_frames", C.c_int32), ("n", C.c_int64 * 3),
                ("origin", C.c_double * 3), ("spacing", C.c_double * 3),
                ("periodic_mask", C.c_uint32), ("frames_f32", C.c_uint32),
                ("t_first", C.c_double), ("dt_frame", C.c_double),
                ("u", C.c_void_p * 3)]


class _Seeds(C.Structure):
    _fields_ = [("dim", C.c_int32), ("periodic_mask", C.c_uint32), ("n", C.c_int64 * 3),
                ("origin", C.c_double * 3), ("spacing", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        I64 = C.c_int64
        D = C.c_double
        sig = {
            "orc_cell_index_many": (None, [P, P, I64, P]),
            "orc_in_domain": (C.c_int, [P, P]),
            "orc_velocity_at_many": (None, [P, P, P, I64, P]),
            "orc_advect_points": (None, [P, P, P, I64, D, D, P, P, P, P, C.c_int]),
            "orc_advect_seeds": (None, [P, P, P, I64, D, D, D, P, P, P, P, C.c_int]),
            "orc_advect_points_traj": (None, [P, P, P, I64, D, D, P, P, C.c_int]),
            "orc_seed_points": (None, [P, P, I64, P]),
            "orc_cg_point": (None, [P, P, P, P, P, P]),
            "orc_cg_tensor": (None, [P, P, P, P, P, C.c_int]),
            "orc_lambda_max": (D, [C.c_int, P]),
            "orc_ftle": (None, [C.c_int, I64, P, D, P, P, C.c_int]),
            "orc_max_threads": (C.c_int, []),
            "orc_aux_points": (None, [P, P, I64, P, P]),
            "orc_eig_many": (None, [C.c_int, I64, P, P, P]),
            "orc_advect_seeds_snap": (None, [P, P, P, I64, D, D, C.c_int, P, P, P, P, C.c_int]),
            "orc_ftle_early": (None, [P, P, P, I64, D, D, P, P, P, P, C.c_int]),
            "orc_cg_aux": (None, [C.c_int, I64, P, P, P, P, P]),
            "orc_advect_seeds_ab": (None, [P, P, P, I64, D, D, D, C.c_int, P, P, P, P, C.c_int]),
            "orc_advect_points_ab": (None, [P, P, P, I64, D, D, C.c_int, P, P, P, P, C.c_int]),
            "orc_mesh_new": (P, [C.c_int32, I64, P, I64, P, C.c_int32, D, D, P]),
            "orc_mesh_free": (None, [P]),
            "orc_mesh_locate_many": (None, [P, P, I64, P, P]),
            "orc_mesh_velocity_at_many": (None, [P, P, P, I64, P, P]),
            "orc_mesh_advect_seeds": (None, [P, P, P, I64, D, D, D, P, P, P, P, P, C.c_int]),
            "orc_mesh_advect_points": (None, [P, P, P, I64, D, D, P, P, P, P, P, C.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


class Velocity:
    """Holds FP64 copies of the frames and the descriptor the C code reads."""

    def __init__(self, fs, keep_f32: bool = False):
        """keep_f32: read FP32 frames in place (each value widened to FP64 when
        used) instead of making an FP64 copy -- for very large frame sets."""
        self.dim = fs.dim
        f32 = keep_f32 and all(np.asarray(c).dtype == np.float32 for c in fs.u)
        dt = np.float32 if f32 else np.float64
        self._u = [np.ascontiguousarray(c, dtype=dt) for c in fs.u]
        s = _Vel()
        s.dim = fs.dim
        s.n_frames = fs.n_frames
        for a in range(3):
            s.n[a] = int(fs.n[a])
            s.origin[a] = float(fs.origin[a])
            s.spacing[a] = float(fs.spacing[a])
        s.periodic_mask = int(fs.periodic_mask)
        s.frames_f32 = 1 if f32 else 0
        s.t_first = float(fs.t_first)
        s.dt_frame = float(fs.dt_frame)
        for c in range(3):
            s.u[c] = self._u[c].ctypes.data if c < fs.dim else None
        self.s = s
        self.fs = fs

    @property
    def ref(self):
        return C.byref(self.s)


def _seeds(g) -> _Seeds:
    s = _Seeds()
    s.dim = g.dim
    s.periodic_mask = int(g.periodic_mask)
    for a in range(3):
        s.n[a] = int(g.n[a])
        s.origin[a] = float(g.origin[a])
        s.spacing[a] = float(g.spacing[a])
    return s


def velocity_at(vel: Velocity, x: np.ndarray, t) -> np.ndarray:
    """u(x, t) at points x (dim x m); t scalar or (m,)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    m = x.shape[1]
    tt = np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64), (m,)))
    out = np.empty_like(x)
    lib().orc_velocity_at_many(vel.ref, _ptr(x), _ptr(tt), m, _ptr(out))
    return out


def in_domain(vel: Velocity, x: Sequence[float]) -> bool:
    q = np.zeros(3)
    q[: vel.dim] = x
    return bool(lib().orc_in_domain(vel.ref, _ptr(q)))


def cell_index(vel: Velocity, x: np.ndarray) -> np.ndarray:
    """Velocity-cell index of positions x (dim x m), computed in FP64."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    m = x.shape[1]
    out = np.empty(m, dtype=np.int64)
    lib().orc_cell_index_many(vel.ref, _ptr(x), m, _ptr(out))
    return out


def advect_points(vel: Velocity, x0: np.ndarray, t0, T: float, dt: float, threads=None,
                  margin: bool = False):
    """RK4 flow map of arbitrary points; returns (xf, cell, flags[, margin])."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    m = x0.shape[1]
    tt = np.ascontiguousarray(np.broadcast_to(np.asarray(t0, dtype=np.float64), (m,)))
    xf = np.empty_like(x0)
    cell = np.empty(m, dtype=np.int64)
    flags = np.empty(m, dtype=np.uint8)
    mg = np.empty(m) if margin else None
    lib().orc_advect_points(vel.ref, _ptr(x0), _ptr(tt), m, float(T), float(dt), _ptr(xf),
                            _ptr(cell), _ptr(flags), _ptr(mg), threads or default_threads())
    return (xf, cell, flags, mg) if margin else (xf, cell, flags)


def advect_points_traj(vel: Velocity, x0: np.ndarray, t0, T: float, dt: float, threads=None):
    """Positions after every step: array (N, dim, m); plus flags."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    m = x0.shape[1]
    tt = np.ascontiguousarray(np.broadcast_to(np.asarray(t0, dtype=np.float64), (m,)))
    N = int(round(T / dt))
    traj = np.empty((N, vel.dim, m), dtype=np.float64)
    flags = np.empty(m, dtype=np.uint8)
    lib().orc_advect_points_traj(vel.ref, _ptr(x0), _ptr(tt), m, float(T), float(dt),
                                 _ptr(traj), _ptr(flags), threads or default_threads())
    return traj, flags


def seed_points(g, idx: Optional[np.ndarray] = None) -> np.ndarray:
    """FP64 positions of the seeds with linear indices idx (all seeds if None)."""
    if idx is None:
        idx = np.arange(g.count, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((g.dim, idx.size), dtype=np.float64)
    sg = _seeds(g)
    lib().orc_seed_points(C.byref(sg), _ptr(idx), idx.size, _ptr(out))
    return out


def advect_seeds(vel: Velocity, g, t0: float, T: float, dt: float, idx=None, threads=None,
                 margin: bool = False):
    """RK4 flow map of the seed grid (or of the seeds idx); returns (xf, cell, flags[, margin])."""
    sg = _seeds(g)
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        m = idx.size
    else:
        m = g.count
    xf = np.empty((g.dim, m), dtype=np.float64)
    cell = np.empty(m, dtype=np.int64)
    flags = np.empty(m, dtype=np.uint8)
    mg = np.empty(m) if margin else None
    lib().orc_advect_seeds(vel.ref, C.byref(sg), _ptr(idx), m, float(t0), float(T), float(dt),
                           _ptr(xf), _ptr(cell), _ptr(flags), _ptr(mg), threads or default_threads())
    return (xf, cell, flags, mg) if margin else (xf, cell, flags)


def aux_points(g, delta, idx=None) -> np.ndarray:
    """Auxiliary points x0 -+ delta_b e_b of the seeds idx (all if None):
    array (dim, 2*dim*m), point q = 2b + side of seed p at column q*m + p."""
    sg = _seeds(g)
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        m = idx.size
    else:
        m = g.count
    dl = np.zeros(3)
    dl[: g.dim] = delta
    x = np.empty((g.dim, 2 * g.dim * m))
    lib().orc_aux_points(C.byref(sg), _ptr(idx), m, _ptr(dl), _ptr(x))
    return x


def cg_aux(dim: int, delta, xf: np.ndarray, flags: Optional[np.ndarray] = None):
    """(C (nq x m), stencil flags (m,)) from the final auxiliary positions
    xf (dim, 2*dim*m) laid out as aux_points returns them."""
    xf = np.ascontiguousarray(xf, dtype=np.float64)
    m = xf.shape[1] // (2 * dim)
    dl = np.zeros(3)
    dl[:dim] = delta
    Cm = np.empty((dim * (dim + 1) // 2, m))
    sfl = np.empty(m, dtype=np.uint8)
    if flags is not None:
        flags = np.ascontiguousarray(flags, dtype=np.uint8)
    lib().orc_cg_aux(dim, m, _ptr(dl), _ptr(xf), _ptr(flags), _ptr(Cm), _ptr(sfl))
    return Cm, sfl


def advect_aux(vel: Velocity, g, delta, t0: float, T: float, dt: float, idx=None, threads=None):
    """Auxiliary-point flow map and C: (xf_aux, flags_aux, margin_aux, C, sflags)."""
    x = aux_points(g, delta, idx)
    xf, _, flags, mg = advect_points(vel, x, t0, T, dt, threads=threads, margin=True)
    Cm, sfl = cg_aux(g.dim, delta, xf, flags)
    return xf, flags, mg, Cm, sfl


def advect_seeds_ab(vel: Velocity, g, t0: float, T: float, dt: float, order: int = 4, idx=None,
                    threads=None, margin: bool = False):
    """Adams-Bashforth (order 2-4, RK4 start-up) flow map of the seed grid:
    (xf, cell, flags[, margin])."""
    assert order in (2, 3, 4)
    sg = _seeds(g)
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        m = idx.size
    else:
        m = g.count
    xf = np.empty((g.dim, m), dtype=np.float64)
    cell = np.empty(m, dtype=np.int64)
    flags = np.empty(m, dtype=np.uint8)
    mg = np.empty(m) if margin else None
    lib().orc_advect_seeds_ab(vel.ref, C.byref(sg), _ptr(idx), m, float(t0), float(T), float(dt),
                              int(order), _ptr(xf), _ptr(cell), _ptr(flags), _ptr(mg),
                              threads or default_threads())
    return (xf, cell, flags, mg) if margin else (xf, cell, flags)


def advect_points_ab(vel: Velocity, x0: np.ndarray, t0, T: float, dt: float, order: int = 4,
                     threads=None, margin: bool = False):
    """Adams-Bashforth flow map of arbitrary points: (xf, cell, flags[, margin])."""
    assert order in (2, 3, 4)
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    m = x0.shape[1]
    tt = np.ascontiguousarray(np.broadcast_to(np.asarray(t0, dtype=np.float64), (m,)))
    xf = np.empty_like(x0)
    cell = np.empty(m, dtype=np.int64)
    flags = np.empty(m, dtype=np.uint8)
    mg = np.empty(m) if margin else None
    lib().orc_advect_points_ab(vel.ref, _ptr(x0), _ptr(tt), m, float(T), float(dt), int(order),
                               _ptr(xf), _ptr(cell), _ptr(flags), _ptr(mg),
                               threads or default_threads())
    return (xf, cell, flags, mg) if margin else (xf, cell, flags)


def cg_tensor(g, xf: np.ndarray, flags: Optional[np.ndarray] = None, threads=None):
    """Packed C (nq x Ns) and stencil flags from final positions xf (dim x Ns)."""
    xf = np.ascontiguousarray(xf, dtype=np.float64)
    Ns = g.count
    assert xf.shape == (g.dim, Ns)
    nq = g.dim * (g.dim + 1) // 2
    Cm = np.empty((nq, Ns), dtype=np.float64)
    sfl = np.empty(Ns, dtype=np.uint8)
    if flags is not None:
        flags = np.ascontiguousarray(flags, dtype=np.uint8)
    sg = _seeds(g)
    lib().orc_cg_tensor(C.byref(sg), _ptr(xf), _ptr(flags), _ptr(Cm), _ptr(sfl),
                        threads or default_threads())
    return Cm, sfl


def cg_point(g, ijk, xc, xm, xp) -> np.ndarray:
    """Packed C at one seed from its own and its neighbours' final positions."""
    sg = _seeds(g)
    ijk3 = np.zeros(3, dtype=np.int64)
    ijk3[: g.dim] = ijk
    xc = np.ascontiguousarray(xc, dtype=np.float64)
    xm_arr = [np.ascontiguousarray(xm[b], dtype=np.float64) for b in range(g.dim)]
    xp_arr = [np.ascontiguousarray(xp[b], dtype=np.float64) for b in range(g.dim)]
    pm = (C.c_void_p * 3)(*[a.ctypes.data for a in xm_arr] + [None] * (3 - g.dim))
    pp = (C.c_void_p * 3)(*[a.ctypes.data for a in xp_arr] + [None] * (3 - g.dim))
    out = np.empty(6, dtype=np.float64)
    lib().orc_cg_point(C.byref(sg), _ptr(ijk3), _ptr(xc), pm, pp, _ptr(out))
    return out[: g.dim * (g.dim + 1) // 2]


def lambda_max(dim: int, Cpacked: np.ndarray) -> float:
    c = np.zeros(6)
    c[: dim * (dim + 1) // 2] = Cpacked
    return float(lib().orc_lambda_max(dim, _ptr(c)))


def advect_seeds_snap(vel: Velocity, g, t0: float, dt: float, snap_steps, idx=None,
                      threads=None):
    """Positions after each of snap_steps RK4 steps: (xf (n_snap, dim, m),
    flags (n_snap, m), steps_done (m,))."""
    sg = _seeds(g)
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        m = idx.size
    else:
        m = g.count
    st = np.ascontiguousarray(snap_steps, dtype=np.int64)
    assert st.size >= 1 and st[0] >= 1 and np.all(np.diff(st) > 0)
    xf = np.empty((st.size, g.dim, m))
    fl = np.empty((st.size, m), dtype=np.uint8)
    done = np.empty(m, dtype=np.int64)
    lib().orc_advect_seeds_snap(vel.ref, C.byref(sg), _ptr(idx), m, float(t0), float(dt),
                                int(st.size), _ptr(st), _ptr(xf), _ptr(fl), _ptr(done),
                                threads or default_threads())
    return xf, fl, done


def ftle_early(vel: Velocity, g, t0: float, dt: float, steps_done, idx=None, threads=None):
    """(lambda_max, ftle, t_eff) with early evaluation for seeds whose stencil
    left the domain, at the seeds idx (all if None); steps_done covers every seed."""
    sg = _seeds(g)
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        m = idx.size
    else:
        m = g.count
    done = np.ascontiguousarray(steps_done, dtype=np.int64)
    assert done.size == g.count
    lam = np.empty(m)
    sig = np.empty(m)
    te = np.empty(m)
    lib().orc_ftle_early(vel.ref, C.byref(sg), _ptr(idx), m, float(t0), float(dt), _ptr(done),
                         _ptr(lam), _ptr(sig), _ptr(te), threads or default_threads())
    return lam, sig, te


def eig(dim: int, Cm: np.ndarray):
    """(evals (dim x n) ascending, evecs (dim, dim, n): evecs[k, a] = component a
    of eigenvector k, sign-normalised) of packed symmetric tensors (nq x n)."""
    Cm = np.ascontiguousarray(Cm, dtype=np.float64)
    n = Cm.shape[1]
    ev = np.empty((dim, n))
    V = np.empty((dim, dim, n))
    lib().orc_eig_many(dim, n, _ptr(Cm), _ptr(ev), _ptr(V))
    return ev, V


def ftle(dim: int, Cm: np.ndarray, T: float, threads=None):
    """(lambda_max, ftle) from packed C (nq x Ns)."""
    Cm = np.ascontiguousarray(Cm, dtype=np.float64)
    Ns = Cm.shape[1]
    lam = np.empty(Ns)
    sig = np.empty(Ns)
    lib().orc_ftle(dim, Ns, _ptr(Cm), float(T), _ptr(lam), _ptr(sig), threads or default_threads())
    return lam, sig


# ---------------------------------------------------------------------------
# Unstructured meshes
# ---------------------------------------------------------------------------


class MeshVelocity:
    """FP64 copies of a mesh and its nodal velocity frames, and the C object
    (with its bucket locator) that reads them."""

    def __init__(self, mf):
        mesh = mf.mesh
        self.dim = mesh.dim
        self.mf = mf
        self._nodes = np.ascontiguousarray(mesh.nodes, dtype=np.float64)
        self._cells = np.ascontiguousarray(mesh.cells, dtype=np.int32)
        self._u = np.ascontiguousarray(mf.u, dtype=np.float64)
        assert self._u.shape == (mf.n_frames, mesh.n_nodes, mesh.dim)
        self._h = lib().orc_mesh_new(mesh.dim, mesh.n_nodes, _ptr(self._nodes), mesh.n_cells,
                                     _ptr(self._cells), mf.n_frames, float(mf.t_first),
                                     float(mf.dt_frame), _ptr(self._u))
        if not self._h:
            raise MemoryError("orc_mesh_new failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_mesh_free(h)
            self._h = None

    def locate(self, x: np.ndarray):
        """(cell (m,), barycentric (dim+1, m)) of points x (dim x m); cell -1 outside."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        m = x.shape[1]
        cell = np.empty(m, dtype=np.int64)
        lam = np.empty((self.dim + 1, m))
        lib().orc_mesh_locate_many(self._h, _ptr(x), m, _ptr(cell), _ptr(lam))
        return cell, lam

    def velocity_at(self, x: np.ndarray, t):
        """(u (dim x m), found (m,)) at points x; u is NaN where not found."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        m = x.shape[1]
        tt = np.ascontiguousarray(np.broadcast_to(np.asarray(t, dtype=np.float64), (m,)))
        out = np.empty_like(x)
        found = np.empty(m, dtype=np.uint8)
        lib().orc_mesh_velocity_at_many(self._h, _ptr(x), _ptr(tt), m, _ptr(out), _ptr(found))
        return out, found.astype(bool)

    def advect_seeds(self, g, t0: float, T: float, dt: float, idx=None, threads=None):
        """RK4 flow map of the seed grid on the mesh field: (xf, cell, flags,
        margin, lam_margin); margin = smallest distance of a checked point to
        the mesh bounding box, lam_margin = smallest barycentric coordinate of
        the final position in its cell."""
        sg = _seeds(g)
        if idx is not None:
            idx = np.ascontiguousarray(idx, dtype=np.int64)
            m = idx.size
        else:
            m = g.count
        xf = np.empty((g.dim, m))
        cell = np.empty(m, dtype=np.int64)
        flags = np.empty(m, dtype=np.uint8)
        mg = np.empty(m)
        lm = np.empty(m)
        lib().orc_mesh_advect_seeds(self._h, C.byref(sg), _ptr(idx), m, float(t0), float(T),
                                    float(dt), _ptr(xf), _ptr(cell), _ptr(flags), _ptr(mg),
                                    _ptr(lm), threads or default_threads())
        return xf, cell, flags, mg, lm

    def advect_points(self, x0: np.ndarray, t0, T: float, dt: float, threads=None):
        """RK4 flow map of points x0 (dim x m) with start times t0: as advect_seeds."""
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        m = x0.shape[1]
        tt = np.ascontiguousarray(np.broadcast_to(np.asarray(t0, dtype=np.float64), (m,)))
        xf = np.empty_like(x0)
        cell = np.empty(m, dtype=np.int64)
        flags = np.empty(m, dtype=np.uint8)
        mg = np.empty(m)
        lm = np.empty(m)
        lib().orc_mesh_advect_points(self._h, _ptr(x0), _ptr(tt), m, float(T), float(dt),
                                     _ptr(xf), _ptr(cell), _ptr(flags), _ptr(mg), _ptr(lm),
                                     threads or default_threads())
        return xf, cell, flags, mg, lm
