"""ctypes binding of the C ABI in ``include/lcs.h`` (argument marshalling only).

Every function here has the name of the C entry point it calls.  Buffers are
torch tensors on the GPU (PyTorch provides device memory and streams); all
computation happens in ``liblcs_hip.so``.  There is no fallback: if the HIP
library is missing the import of this module fails.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblcs_hip.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "lcs.h")

LCS_OK = 0
LCS_E_ARG = -1
LCS_E_SHAPE = -2
LCS_E_TIME_RANGE = -3
LCS_E_SEED_DOMAIN = -4
LCS_E_STEP = -5
LCS_E_HIP = -6
LCS_E_UNSUPPORTED = -7

FLAG_OUT = 1
FLAG_NONFINITE = 2
FLAG_STENCIL_OUT = 4
FLAG_TIME_OUT = 8

_STATUS_NAMES = {0: "LCS_OK", -1: "LCS_E_ARG", -2: "LCS_E_SHAPE", -3: "LCS_E_TIME_RANGE",
                 -4: "LCS_E_SEED_DOMAIN", -5: "LCS_E_STEP", -6: "LCS_E_HIP", -7: "LCS_E_UNSUPPORTED"}


class LcsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class lcs_velocity_t(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_frames", C.c_int32), ("n", C.c_int64 * 3),
                ("origin", C.c_double * 3), ("spacing", C.c_double * 3),
                ("periodic_mask", C.c_uint32), ("layout", C.c_uint32),
                ("t_first", C.c_double), ("dt_frame", C.c_double),
                ("u", C.c_void_p * 3)]


class lcs_seed_grid_t(C.Structure):
    _fields_ = [("dim", C.c_int32), ("periodic_mask", C.c_uint32), ("n", C.c_int64 * 3),
                ("origin", C.c_double * 3), ("spacing", C.c_double * 3)]


class lcs_window_t(C.Structure):
    _fields_ = [("t0", C.c_double), ("T", C.c_double)]


def _load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is not built (run __graft_entry__.build())")
    # torch carries its own HIP runtime (same soname as ROCm's).  Loading torch
    # first makes the library bind to that one runtime; loading the library
    # first would put a second HIP/HSA runtime into the process once torch is
    # imported, and one of them then finds no device.
    import torch  # noqa: F401
    L = C.CDLL(path)
    P, D, I64, I32 = C.c_void_p, C.c_double, C.c_int64, C.c_int32
    sig = {
        "lcs_advect": [P, P, D, D, D, P, P, P, P],
        "lcs_advect_points": [P, P, P, I64, D, D, P, P, P, P],
        "lcs_cg_tensor": [P, P, P, P, P, P],
        "lcs_ftle": [I32, I64, P, D, P, P, P],
        "lcs_cg_ftle": [P, P, P, D, P, P, P, P],
        "lcs_sync_status": [P],
        "lcs_timing_enable": [I32],
        "lcs_timing_query": [C.c_char_p, P, P],
        "lcs_advect_batched": [P, P, P, P, I32, D, P, P, P, P],
        "lcs_plan_create": [P, C.c_char_p],
        "lcs_advect_tuned": [P, P, P, D, D, D, P, P, P, P, I64, P, I32, P, P, P],
        "lcs_plan_destroy": [P],
        "lcs_plan_stats": [P, P, P],
        "lcs_mlp_refresh_bf16": [P, P, P],
        "lcs_mlp_forward": [P, P, I64, P, P, I64, I32, P],
        "lcs_mlp_backward": [P, P, P, I64, P, P, I64, P],
        "lcs_mse_grad": [P, P, I64, P, P, P],
        "lcs_adam_step": [P, P, P, P, I64, C.c_float, C.c_float, C.c_float, C.c_float, I32, P],
        "lcs_surrogate_compose": [P, P, D, D, I32, P, P],
        "lcs_surrogate_check": [P, P, D, D, D, P, C.c_float, P, P, P, P],
        "lcs_advect_tiles": [P, P, D, D, D, P, P, P, P, P],
        "lcs_surrogate_flowmap": [P, P, P, D, D, I32, D, D, D, P, P, P, P, P, P, I64, P],
        "lcs_sub": [P, P, I64, P, P],
        "lcs_mlp_train": [P, P, P, P, P, I64, I64, I32, I32, I32, C.c_float, C.c_float,
                          C.c_float, C.c_float, C.c_float, P, P, P, P, P, I64, P],
        "lcs_advect_sorted": [P, P, D, D, D, I32, P, P, P, P, I64, P],
        "lcs_advect_sorted_noalloc": [P, P, D, D, D, I32, P, P, P, P],
        "lcs_advect_ab": [P, P, I32, D, D, D, P, P, P, P],
        "lcs_frames_interleave": [P, C.c_uint32, I32, I32, P, P, P],
        "lcs_advect_aux": [P, P, P, D, D, D, P, P, P, P],
        "lcs_advect_aux_sorted": [P, P, P, D, D, D, I32, P, P, P, P, I64, P],
        "lcs_cg_eig": [I32, I64, P, P, P, P],
        "lcs_advect_ab_sorted": [P, P, I32, D, D, D, I32, P, P, P, P, I64, P],
        "lcs_advect_snapshots": [P, P, D, D, I32, P, P, P, P, P],
        "lcs_ftle_early": [P, P, D, D, I32, P, P, P, P, P, P, I64, P],
        "lcs_cg_aux": [P, P, P, P, P, P, P, P],
        "lcs_mesh_create": [P, P, P],
        "lcs_mesh_info": [P, P],
        "lcs_mesh_locate": [P, P, I64, P, P, P],
        "lcs_mesh_velocity_at": [P, P, P, P, I64, P, P, P],
        "lcs_mesh_advect": [P, P, P, D, D, D, P, P, P, P],
        "lcs_mesh_advect_points": [P, P, P, P, I64, D, D, P, P, P, P],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.restype = C.c_int
        fn.argtypes = args
    L.lcs_mesh_destroy.restype = None
    L.lcs_mesh_destroy.argtypes = [P]
    L.lcs_last_error.restype = C.c_char_p
    L.lcs_last_error.argtypes = []
    L.lcs_version.restype = C.c_int32
    L.lcs_version.argtypes = []
    for name in ("lcs_mlp_workspace_bytes", "lcs_mlp_backward_scratch_bytes"):
        fn = getattr(L, name)
        fn.restype = C.c_int64
    L.lcs_mlp_workspace_bytes.argtypes = [I64, I32]
    L.lcs_advect_sorted_workspace_bytes.restype = C.c_int64
    L.lcs_advect_sorted_workspace_bytes.argtypes = [P, P]
    L.lcs_advect_aux_sorted_workspace_bytes.restype = C.c_int64
    L.lcs_advect_aux_sorted_workspace_bytes.argtypes = [P, P]
    L.lcs_advect_ab_sorted_workspace_bytes.restype = C.c_int64
    L.lcs_advect_ab_sorted_workspace_bytes.argtypes = [P, P]
    L.lcs_ftle_early_workspace_bytes.restype = C.c_int64
    L.lcs_ftle_early_workspace_bytes.argtypes = [P]
    L.lcs_surrogate_flowmap_workspace_bytes.restype = C.c_int64
    L.lcs_surrogate_flowmap_workspace_bytes.argtypes = [P, P, D]
    L.lcs_check_tile_count.restype = C.c_int64
    L.lcs_check_tile_count.argtypes = [P]
    L.lcs_frames_interleave_floats.restype = C.c_int64
    L.lcs_frames_interleave_floats.argtypes = [P, C.c_uint32, I32]
    L.lcs_mlp_backward_scratch_bytes.argtypes = [I64]
    L.lcs_mlp_train_workspace_bytes.restype = C.c_int64
    L.lcs_mlp_train_workspace_bytes.argtypes = [I64]
    return L


_lib = _load()


def lib():
    return _lib


def declared_entry_points() -> list:
    """Names of the functions ``include/lcs.h`` declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lcs_[a-z0-9_]+)\s*\(", text)))


def lcs_last_error() -> str:
    return _lib.lcs_last_error().decode()


def lcs_version() -> int:
    return int(_lib.lcs_version())


def _check(status: int):
    if status != LCS_OK:
        raise LcsError(status, lcs_last_error())


# ---------------------------------------------------------------------------
# Descriptors
# ---------------------------------------------------------------------------


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, dtype, shape, what):
    torch = _torch()
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


class DeviceFrames:
    """Velocity frames resident in HBM (one FP32 tensor per component) and the
    ``lcs_velocity_t`` that describes them."""

    def __init__(self, fs, device="cuda", tensors: Optional[Sequence] = None):
        torch = _torch()
        if tensors is None:
            tensors = [torch.from_numpy(np.ascontiguousarray(c, dtype=np.float32)).to(device)
                       for c in fs.u]
        self.u = list(tensors)
        self.fs = fs
        d = lcs_velocity_t()
        d.dim = fs.dim
        d.n_frames = int(self.u[0].shape[0])
        for a in range(3):
            d.n[a] = int(fs.n[a])
            d.origin[a] = float(fs.origin[a])
            d.spacing[a] = float(fs.spacing[a])
        d.periodic_mask = int(fs.periodic_mask)
        d.layout = LCS_LAYOUT_SOA
        d.t_first = float(fs.t_first)
        d.dt_frame = float(fs.dt_frame)
        nodes = int(fs.n[0] * fs.n[1] * fs.n[2])
        for c in range(3):
            if c < fs.dim:
                t = self.u[c]
                _need(t, torch.float32, t.shape, f"frame component {c}")
                if t.numel() != d.n_frames * nodes:
                    raise ValueError("frame tensor size does not match the grid")
                d.u[c] = t.data_ptr()
            else:
                d.u[c] = None
        self.desc = d

    @property
    def dim(self) -> int:
        return self.desc.dim

    @property
    def ref(self):
        return C.byref(self.desc)

    @classmethod
    def interleaved(cls, fs, layout: str = "xyz", device="cuda", stream=None) -> "DeviceFrames":
        """Frames of the FrameSet fs staged on the device in an interleaved layout
        ("xyz": dim floats per node, "xyzw": 4 in 3D, "tpair": time-paired
        records of 2*dim floats) by lcs_frames_interleave."""
        return lcs_frames_interleave(cls(fs, device=device), layout, stream=stream)


LCS_LAYOUT_SOA, LCS_LAYOUT_XYZ, LCS_LAYOUT_XYZW, LCS_LAYOUT_TPAIR = 0, 1, 2, 3
_LAYOUTS = {"xyz": LCS_LAYOUT_XYZ, "xyzw": LCS_LAYOUT_XYZW, "tpair": LCS_LAYOUT_TPAIR}


class _InterleavedFrames(DeviceFrames):
    """Frames in an interleaved layout: one tensor ((F, N, S), or (F-1, N', 2*dim)
    for time-paired records) and its descriptor."""

    def __init__(self, fs, tensor, desc):     # noqa: D401 (no SoA construction)
        self.fs = fs
        self.u = [tensor]
        self.desc = desc


def lcs_frames_interleave(frames: DeviceFrames, layout: str = "xyz", f_first: int = 0,
                          f_count: Optional[int] = None, out=None, stream=None) -> DeviceFrames:
    """Copy (a span of) structure-of-arrays frames into the interleaved layout."""
    torch = _torch()
    lay = _LAYOUTS[layout]
    d = frames.desc
    F = int(d.n_frames) if f_count is None else int(f_count)
    if lay == LCS_LAYOUT_TPAIR:
        shape = (F - 1, int((d.n[0] + 1) * d.n[1] * d.n[2]), 2 * int(d.dim))
    else:
        shape = (F, int(d.n[0] * d.n[1] * d.n[2]), 4 if lay == LCS_LAYOUT_XYZW else int(d.dim))
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=frames.u[0].device)
    _need(out, torch.float32, shape, "out")
    nd = lcs_velocity_t()
    _check(_lib.lcs_frames_interleave(frames.ref, lay, int(f_first), F, _ptr(out), C.byref(nd),
                                      _stream_handle(stream)))
    return _InterleavedFrames(frames.fs, out, nd)


def seed_grid_desc(g) -> lcs_seed_grid_t:
    s = lcs_seed_grid_t()
    s.dim = g.dim
    s.periodic_mask = int(g.periodic_mask)
    for a in range(3):
        s.n[a] = int(g.n[a])
        s.origin[a] = float(g.origin[a])
        s.spacing[a] = float(g.spacing[a])
    return s


# ---------------------------------------------------------------------------
# Entry points
# ---------------------------------------------------------------------------


def lcs_advect(frames: DeviceFrames, seeds, t0: float, T: float, dt: float,
               xf=None, cell=None, flags=None, want_cell=True, want_flags=True, stream=None):
    """Flow map of the seed grid; returns (xf [dim,Ns] f32, cell [Ns] i64, flags [Ns] u8)."""
    torch = _torch()
    dev = frames.u[0].device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    d = seeds.dim
    if xf is None:
        xf = torch.empty((d, ns), dtype=torch.float32, device=dev)
    if cell is None and want_cell:
        cell = torch.empty(ns, dtype=torch.int64, device=dev)
    if flags is None and want_flags:
        flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    _need(xf, torch.float32, (d, ns), "xf")
    _need(cell, torch.int64, (ns,), "cell")
    _need(flags, torch.uint8, (ns,), "flags")
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_advect(frames.ref, C.byref(sd), float(t0), float(T), float(dt),
                           _ptr(xf), _ptr(cell), _ptr(flags), _stream_handle(stream)))
    return xf, cell, flags


def lcs_advect_ab(frames: DeviceFrames, seeds, t0: float, T: float, dt: float, order: int = 4,
                  xf=None, cell=None, flags=None, want_cell=True, want_flags=True, stream=None):
    """Adams-Bashforth (order 2-4, RK4 start-up) flow map of a seed grid."""
    torch = _torch()
    dev = frames.u[0].device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    d = seeds.dim
    if xf is None:
        xf = torch.empty((d, ns), dtype=torch.float32, device=dev)
    if cell is None and want_cell:
        cell = torch.empty(ns, dtype=torch.int64, device=dev)
    if flags is None and want_flags:
        flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    _need(xf, torch.float32, (d, ns), "xf")
    _need(cell, torch.int64, (ns,), "cell")
    _need(flags, torch.uint8, (ns,), "flags")
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_advect_ab(frames.ref, C.byref(sd), int(order), float(t0), float(T), float(dt),
                              _ptr(xf), _ptr(cell), _ptr(flags), _stream_handle(stream)))
    return xf, cell, flags


def lcs_advect_aux(frames: DeviceFrames, seeds, delta, t0: float, T: float, dt: float,
                   xa_hi=None, xa_lo=None, flags=None, want_flags=True, stream=None):
    """Flow map of the 2*dim auxiliary points x0 -+ delta_b e_b of every seed:
    (xa_hi, xa_lo, flags), positions [dim][2*dim][Ns] as two-floats."""
    torch = _torch()
    dev = frames.u[0].device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    d = seeds.dim
    if xa_hi is None:
        xa_hi = torch.empty((d, 2 * d, ns), dtype=torch.float32, device=dev)
    if xa_lo is None:
        xa_lo = torch.empty((d, 2 * d, ns), dtype=torch.float32, device=dev)
    if flags is None and want_flags:
        flags = torch.empty((2 * d, ns), dtype=torch.uint8, device=dev)
    _need(xa_hi, torch.float32, (d, 2 * d, ns), "xa_hi")
    _need(xa_lo, torch.float32, (d, 2 * d, ns), "xa_lo")
    _need(flags, torch.uint8, (2 * d, ns), "flags")
    dl = (C.c_double * 3)(*([float(x) for x in delta] + [0.0] * (3 - len(delta))))
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_advect_aux(frames.ref, C.byref(sd), dl, float(t0), float(T), float(dt),
                               _ptr(xa_hi), _ptr(xa_lo), _ptr(flags), _stream_handle(stream)))
    return xa_hi, xa_lo, flags


def lcs_advect_aux_sorted_workspace_bytes(frames: DeviceFrames, seeds) -> int:
    sd = seed_grid_desc(seeds)
    return int(_lib.lcs_advect_aux_sorted_workspace_bytes(frames.ref, C.byref(sd)))


def lcs_advect_aux_sorted(frames: DeviceFrames, seeds, delta, t0: float, T: float, dt: float,
                          segment_steps: int = 50, xa_hi=None, xa_lo=None, flags=None,
                          workspace=None, want_flags=True, stream=None):
    """lcs_advect_aux with the auxiliary tracers re-bundled by position between
    segments (same outputs, bit for bit)."""
    torch = _torch()
    dev = frames.u[0].device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    d = seeds.dim
    if xa_hi is None:
        xa_hi = torch.empty((d, 2 * d, ns), dtype=torch.float32, device=dev)
    if xa_lo is None:
        xa_lo = torch.empty((d, 2 * d, ns), dtype=torch.float32, device=dev)
    if flags is None and want_flags:
        flags = torch.empty((2 * d, ns), dtype=torch.uint8, device=dev)
    _need(xa_hi, torch.float32, (d, 2 * d, ns), "xa_hi")
    _need(xa_lo, torch.float32, (d, 2 * d, ns), "xa_lo")
    _need(flags, torch.uint8, (2 * d, ns), "flags")
    if workspace is None:
        workspace = _bytes_buffer(lcs_advect_aux_sorted_workspace_bytes(frames, seeds), dev)
    dl = (C.c_double * 3)(*([float(x) for x in delta] + [0.0] * (3 - len(delta))))
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_advect_aux_sorted(frames.ref, C.byref(sd), dl, float(t0), float(T), float(dt),
                                      int(segment_steps), _ptr(xa_hi), _ptr(xa_lo), _ptr(flags),
                                      _ptr(workspace), int(workspace.numel()),
                                      _stream_handle(stream)))
    return xa_hi, xa_lo, flags


def lcs_cg_aux(seeds, delta, xa_hi, xa_lo, flags=None, C_out=None, stencil_flags=None,
               want_stencil=True, stream=None):
    """C (packed, FP64) and stencil flags from auxiliary-point positions."""
    torch = _torch()
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    d = seeds.dim
    dev = xa_hi.device
    _need(xa_hi, torch.float32, (d, 2 * d, ns), "xa_hi")
    _need(xa_lo, torch.float32, (d, 2 * d, ns), "xa_lo")
    _need(flags, torch.uint8, (2 * d, ns), "flags")
    nq = d * (d + 1) // 2
    if C_out is None:
        C_out = torch.empty((nq, ns), dtype=torch.float64, device=dev)
    if stencil_flags is None and want_stencil:
        stencil_flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    _need(C_out, torch.float64, (nq, ns), "C")
    _need(stencil_flags, torch.uint8, (ns,), "stencil_flags")
    dl = (C.c_double * 3)(*([float(x) for x in delta] + [0.0] * (3 - len(delta))))
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_cg_aux(C.byref(sd), dl, _ptr(xa_hi), _ptr(xa_lo), _ptr(flags), _ptr(C_out),
                           _ptr(stencil_flags), _stream_handle(stream)))
    return C_out, stencil_flags


def lcs_advect_ab_sorted_workspace_bytes(frames: DeviceFrames, seeds) -> int:
    sd = seed_grid_desc(seeds)
    return int(_lib.lcs_advect_ab_sorted_workspace_bytes(frames.ref, C.byref(sd)))


def lcs_advect_ab_sorted(frames: DeviceFrames, seeds, t0: float, T: float, dt: float,
                         order: int = 4, segment_steps: int = 0, xf=None, cell=None, flags=None,
                         workspace=None, want_cell=True, want_flags=True, stream=None):
    """lcs_advect_ab with tracers re-bundled by position between segments."""
    torch = _torch()
    dev = frames.u[0].device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    d = seeds.dim
    if xf is None:
        xf = torch.empty((d, ns), dtype=torch.float32, device=dev)
    if cell is None and want_cell:
        cell = torch.empty(ns, dtype=torch.int64, device=dev)
    if flags is None and want_flags:
        flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    _need(xf, torch.float32, (d, ns), "xf")
    _need(cell, torch.int64, (ns,), "cell")
    _need(flags, torch.uint8, (ns,), "flags")
    if workspace is None:
        workspace = _bytes_buffer(lcs_advect_ab_sorted_workspace_bytes(frames, seeds), dev)
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_advect_ab_sorted(frames.ref, C.byref(sd), int(order), float(t0), float(T),
                                     float(dt), int(segment_steps), _ptr(xf), _ptr(cell),
                                     _ptr(flags), _ptr(workspace),
                                     int(workspace.numel() * workspace.element_size()),
                                     _stream_handle(stream)))
    return xf, cell, flags


def lcs_cg_eig(dim: int, C_in, evals=None, evecs=None, want_vectors=True, stream=None):
    """(evals (dim, n) ascending, evecs (dim, dim, n)) of packed C (nq, n), FP64."""
    torch = _torch()
    nq = dim * (dim + 1) // 2
    n = int(C_in.shape[1])
    _need(C_in, torch.float64, (nq, n), "C")
    if evals is None:
        evals = torch.empty((dim, n), dtype=torch.float64, device=C_in.device)
    if evecs is None and want_vectors:
        evecs = torch.empty((dim, dim, n), dtype=torch.float64, device=C_in.device)
    _need(evals, torch.float64, (dim, n), "evals")
    _need(evecs, torch.float64, (dim, dim, n), "evecs")
    _check(_lib.lcs_cg_eig(int(dim), n, _ptr(C_in), _ptr(evals), _ptr(evecs), _stream_handle(stream)))
    return evals, evecs


def lcs_advect_snapshots(frames: DeviceFrames, seeds, t0: float, dt: float, snap_steps, xf=None,
                         flags=None, steps_done=None, want_flags=True, want_steps=True,
                         stream=None):
    """Positions (n_snap, dim, Ns), flags (n_snap, Ns) and accepted steps (Ns) after
    each of snap_steps RK4 steps."""
    torch = _torch()
    dev = frames.u[0].device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    d = seeds.dim
    st = [int(x) for x in snap_steps]
    k = len(st)
    if xf is None:
        xf = torch.empty((k, d, ns), dtype=torch.float32, device=dev)
    if flags is None and want_flags:
        flags = torch.empty((k, ns), dtype=torch.uint8, device=dev)
    if steps_done is None and want_steps:
        steps_done = torch.empty(ns, dtype=torch.int32, device=dev)
    _need(xf, torch.float32, (k, d, ns), "xf")
    _need(flags, torch.uint8, (k, ns), "flags")
    _need(steps_done, torch.int32, (ns,), "steps_done")
    arr = (C.c_int32 * k)(*st)
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_advect_snapshots(frames.ref, C.byref(sd), float(t0), float(dt), k, arr,
                                     _ptr(xf), _ptr(flags), _ptr(steps_done),
                                     _stream_handle(stream)))
    return xf, flags, steps_done


def lcs_ftle_early_workspace_bytes(seeds) -> int:
    sd = seed_grid_desc(seeds)
    return int(_lib.lcs_ftle_early_workspace_bytes(C.byref(sd)))


def lcs_ftle_early(frames: DeviceFrames, seeds, t0: float, dt: float, nsteps: int, xf, steps_done,
                   lambda_max=None, ftle=None, t_eff=None, workspace=None, stream=None):
    """FTLE with early evaluation where a stencil left the domain: (lambda_max, ftle, t_eff)."""
    torch = _torch()
    dev = xf.device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    d = seeds.dim
    _need(xf, torch.float32, (d, ns), "xf")
    _need(steps_done, torch.int32, (ns,), "steps_done")
    if lambda_max is None:
        lambda_max = torch.empty(ns, dtype=torch.float64, device=dev)
    if ftle is None:
        ftle = torch.empty(ns, dtype=torch.float64, device=dev)
    if t_eff is None:
        t_eff = torch.empty(ns, dtype=torch.float64, device=dev)
    for t, nm in ((lambda_max, "lambda_max"), (ftle, "ftle"), (t_eff, "t_eff")):
        _need(t, torch.float64, (ns,), nm)
    if workspace is None:
        workspace = _bytes_buffer(lcs_ftle_early_workspace_bytes(seeds), dev)
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_ftle_early(frames.ref, C.byref(sd), float(t0), float(dt), int(nsteps), _ptr(xf),
                               _ptr(steps_done), _ptr(lambda_max), _ptr(ftle), _ptr(t_eff),
                               _ptr(workspace), int(workspace.numel() * workspace.element_size()),
                               _stream_handle(stream)))
    return lambda_max, ftle, t_eff


def lcs_advect_sorted_workspace_bytes(frames: DeviceFrames, seeds) -> int:
    sd = seed_grid_desc(seeds)
    return int(_lib.lcs_advect_sorted_workspace_bytes(frames.ref, C.byref(sd)))


def lcs_advect_sorted(frames: DeviceFrames, seeds, t0: float, T: float, dt: float,
                      segment_steps: int = 0, xf=None, cell=None, flags=None, workspace=None,
                      want_cell=True, want_flags=True, stream=None):
    """lcs_advect with tracers re-bundled by position between segments."""
    torch = _torch()
    dev = frames.u[0].device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    d = seeds.dim
    if xf is None:
        xf = torch.empty((d, ns), dtype=torch.float32, device=dev)
    if cell is None and want_cell:
        cell = torch.empty(ns, dtype=torch.int64, device=dev)
    if flags is None and want_flags:
        flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    _need(xf, torch.float32, (d, ns), "xf")
    _need(cell, torch.int64, (ns,), "cell")
    _need(flags, torch.uint8, (ns,), "flags")
    if workspace is None:
        workspace = _bytes_buffer(lcs_advect_sorted_workspace_bytes(frames, seeds), dev)
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_advect_sorted(frames.ref, C.byref(sd), float(t0), float(T), float(dt),
                                  int(segment_steps), _ptr(xf), _ptr(cell), _ptr(flags),
                                  _ptr(workspace), int(workspace.numel() * workspace.element_size()),
                                  _stream_handle(stream)))
    return xf, cell, flags


LCS_NOALLOC_SCRATCH_BYTES = 64 << 20


def lcs_advect_sorted_noalloc(frames: DeviceFrames, seeds, t0: float, T: float, dt: float,
                              segment_steps: int, xf, cell=None, flags=None, stream=None):
    """lcs_advect_sorted with the library's fixed device scratch as workspace
    (nothing is allocated by the call; xf / cell / flags are the caller's)."""
    torch = _torch()
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    d = seeds.dim
    _need(xf, torch.float32, (d, ns), "xf")
    _need(cell, torch.int64, (ns,), "cell")
    _need(flags, torch.uint8, (ns,), "flags")
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_advect_sorted_noalloc(frames.ref, C.byref(sd), float(t0), float(T), float(dt),
                                          int(segment_steps), _ptr(xf), _ptr(cell), _ptr(flags),
                                          _stream_handle(stream)))
    return xf, cell, flags


def lcs_advect_points(frames: DeviceFrames, x0, t0, T: float, dt: float,
                      xf=None, cell=None, flags=None, want_cell=True, want_flags=True, stream=None):
    """Flow map of points x0 [dim,n] (f32) with start times t0 [n] (f64)."""
    torch = _torch()
    d, n = int(x0.shape[0]), int(x0.shape[1])
    dev = x0.device
    if not isinstance(t0, torch.Tensor):
        t0 = torch.full((n,), float(t0), dtype=torch.float64, device=dev)
    if xf is None:
        xf = torch.empty((d, n), dtype=torch.float32, device=dev)
    if cell is None and want_cell:
        cell = torch.empty(n, dtype=torch.int64, device=dev)
    if flags is None and want_flags:
        flags = torch.empty(n, dtype=torch.uint8, device=dev)
    if d != frames.dim:
        raise ValueError("x0 dimension does not match the frames")
    _need(x0, torch.float32, (d, n), "x0")
    _need(t0, torch.float64, (n,), "t0")
    _need(xf, torch.float32, (d, n), "xf")
    _need(cell, torch.int64, (n,), "cell")
    _need(flags, torch.uint8, (n,), "flags")
    _check(_lib.lcs_advect_points(frames.ref, _ptr(x0), _ptr(t0), n, float(T), float(dt),
                                  _ptr(xf), _ptr(cell), _ptr(flags), _stream_handle(stream)))
    return xf, cell, flags


def lcs_cg_tensor(seeds, xf, flags=None, C_out=None, stencil_flags=None, want_stencil=True,
                  stream=None):
    """Packed Cauchy-Green tensor [nq, Ns] (f64) and stencil flags [Ns] (u8)."""
    torch = _torch()
    d = seeds.dim
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    nq = d * (d + 1) // 2
    dev = xf.device
    if C_out is None:
        C_out = torch.empty((nq, ns), dtype=torch.float64, device=dev)
    if stencil_flags is None and want_stencil:
        stencil_flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    _need(xf, torch.float32, (d, ns), "xf")
    _need(flags, torch.uint8, (ns,), "flags")
    _need(C_out, torch.float64, (nq, ns), "C")
    _need(stencil_flags, torch.uint8, (ns,), "stencil_flags")
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_cg_tensor(C.byref(sd), _ptr(xf), _ptr(flags), _ptr(C_out), _ptr(stencil_flags),
                              _stream_handle(stream)))
    return C_out, stencil_flags


def lcs_ftle(dim: int, C_in, T: float, lambda_max=None, ftle=None, want_lambda=True, stream=None):
    """(lambda_max [n], ftle [n]) in f64 from packed C [nq, n]."""
    torch = _torch()
    nq = dim * (dim + 1) // 2
    n = int(C_in.shape[1])
    dev = C_in.device
    if lambda_max is None and want_lambda:
        lambda_max = torch.empty(n, dtype=torch.float64, device=dev)
    if ftle is None:
        ftle = torch.empty(n, dtype=torch.float64, device=dev)
    _need(C_in, torch.float64, (nq, n), "C")
    _need(lambda_max, torch.float64, (n,), "lambda_max")
    _need(ftle, torch.float64, (n,), "ftle")
    _check(_lib.lcs_ftle(int(dim), n, _ptr(C_in), float(T), _ptr(lambda_max), _ptr(ftle),
                         _stream_handle(stream)))
    return lambda_max, ftle


def lcs_cg_ftle(seeds, xf, T: float, flags=None, lambda_max=None, ftle=None, stencil_flags=None,
                want_lambda=True, want_stencil=True, stream=None):
    """Fused gradient -> C -> lambda_max -> FTLE without materialising C."""
    torch = _torch()
    d = seeds.dim
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    dev = xf.device
    if lambda_max is None and want_lambda:
        lambda_max = torch.empty(ns, dtype=torch.float64, device=dev)
    if ftle is None:
        ftle = torch.empty(ns, dtype=torch.float64, device=dev)
    if stencil_flags is None and want_stencil:
        stencil_flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    _need(xf, torch.float32, (d, ns), "xf")
    _need(flags, torch.uint8, (ns,), "flags")
    _need(lambda_max, torch.float64, (ns,), "lambda_max")
    _need(ftle, torch.float64, (ns,), "ftle")
    _need(stencil_flags, torch.uint8, (ns,), "stencil_flags")
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_cg_ftle(C.byref(sd), _ptr(xf), _ptr(flags), float(T), _ptr(lambda_max),
                            _ptr(ftle), _ptr(stencil_flags), _stream_handle(stream)))
    return lambda_max, ftle, stencil_flags


def lcs_timing_enable(on: bool = True):
    """Record HIP events around every launch of the library's main kernels."""
    _check(_lib.lcs_timing_enable(1 if on else 0))


def lcs_timing_query(kernel: str):
    """(launches, total ms) of the recorded launches of ``kernel`` (after the
    recorded work has completed)."""
    n, ms = C.c_int64(), C.c_double()
    _check(_lib.lcs_timing_query(kernel.encode(), C.byref(n), C.byref(ms)))
    return int(n.value), float(ms.value)


def lcs_sync_status(stream=None):
    _check(_lib.lcs_sync_status(_stream_handle(stream)))


LCS_MAX_WINDOWS = 192


class Plan:
    """Owns an ``lcs_plan_t`` (work counter, capture stream, cached graph, the
    autotuner's choices; ``autotune_cache`` names the file they persist in)."""

    def __init__(self, autotune_cache: Optional[str] = None):
        h = C.c_void_p()
        _check(_lib.lcs_plan_create(C.byref(h),
                                    autotune_cache.encode() if autotune_cache else None))
        self.handle = h

    def stats(self):
        a, b = C.c_int64(), C.c_int64()
        _check(_lib.lcs_plan_stats(self.handle, C.byref(a), C.byref(b)))
        return {"graph_launches": a.value, "graph_captures": b.value}

    def close(self):
        if self.handle is not None and self.handle.value:
            _lib.lcs_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lcs_advect_tuned(plan: Plan, frames: DeviceFrames, seeds, t0: float, T: float, dt: float,
                     xf=None, cell=None, flags=None, workspace=None, candidates=None,
                     want_cell=True, want_flags=True, stream=None):
    """lcs_advect with the plan's autotuned seed ordering.  Returns (xf, cell,
    flags, chosen segment length, {candidate: ms} on a tuning call else None)."""
    torch = _torch()
    dev = frames.u[0].device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    d = seeds.dim
    if xf is None:
        xf = torch.empty((d, ns), dtype=torch.float32, device=dev)
    if cell is None and want_cell:
        cell = torch.empty(ns, dtype=torch.int64, device=dev)
    if flags is None and want_flags:
        flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    _need(xf, torch.float32, (d, ns), "xf")
    _need(cell, torch.int64, (ns,), "cell")
    _need(flags, torch.uint8, (ns,), "flags")
    cand = None if candidates is None else [int(c) for c in candidates]
    nc = 5 if cand is None else len(cand)
    carr = None if cand is None else (C.c_int32 * nc)(*cand)
    ms = (C.c_float * nc)(*([float("nan")] * nc))
    chosen = C.c_int32(-1)
    sd = seed_grid_desc(seeds)
    wsb = 0 if workspace is None else int(workspace.numel() * workspace.element_size())
    _check(_lib.lcs_advect_tuned(plan.handle, frames.ref, C.byref(sd), float(t0), float(T),
                                 float(dt), _ptr(xf), _ptr(cell), _ptr(flags), _ptr(workspace), wsb,
                                 carr, nc if cand is not None else 0, C.byref(chosen), ms,
                                 _stream_handle(stream)))
    tuned = None
    if any(x == x for x in ms):          # a tuning call fills the times (NaN = skipped)
        names = cand if cand is not None else [0, 200, 100, 50, 25]
        tuned = {int(c): (None if v != v else float(v)) for c, v in zip(names, ms)}
    return xf, cell, flags, int(chosen.value), tuned


def lcs_advect_batched(plan: Plan, frames: DeviceFrames, seeds, windows, dt: float,
                       xf=None, cell=None, flags=None, want_cell=True, want_flags=True,
                       stream=None):
    """All windows ((t0, T) pairs) in one graph-replayed persistent launch.
    Returns xf [nw, dim, Ns] f32, cell [nw, Ns] i64, flags [nw, Ns] u8."""
    torch = _torch()
    win = np.ascontiguousarray(np.asarray(windows, dtype=np.float64).reshape(-1, 2))
    nw = int(win.shape[0])
    dev = frames.u[0].device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    d = seeds.dim
    if xf is None:
        xf = torch.empty((nw, d, ns), dtype=torch.float32, device=dev)
    if cell is None and want_cell:
        cell = torch.empty((nw, ns), dtype=torch.int64, device=dev)
    if flags is None and want_flags:
        flags = torch.empty((nw, ns), dtype=torch.uint8, device=dev)
    _need(xf, torch.float32, (nw, d, ns), "xf")
    _need(cell, torch.int64, (nw, ns), "cell")
    _need(flags, torch.uint8, (nw, ns), "flags")
    arr = (lcs_window_t * nw)(*[lcs_window_t(float(a), float(b)) for a, b in win])
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_advect_batched(plan.handle, frames.ref, C.byref(sd), arr, nw, float(dt),
                                   _ptr(xf), _ptr(cell), _ptr(flags), _stream_handle(stream)))
    return xf, cell, flags


# ---------------------------------------------------------------------------
# Learned surrogate (Fourier-feature MLP)
# ---------------------------------------------------------------------------

LCS_MLP_FREQ = 64
LCS_MLP_WIDTH = 256
LCS_MLP_HIDDEN = 4
LCS_MLP_PARAMS = 231171
LCS_MLP_BF16 = 458752


class lcs_mlp_t(C.Structure):
    _fields_ = [("freq", C.c_void_p), ("in_shift", C.c_float * 4), ("in_scale", C.c_float * 4),
                ("out_scale", C.c_float), ("reserved", C.c_uint32), ("params", C.c_void_p),
                ("params_bf16", C.c_void_p)]


class Mlp:
    """Device-resident surrogate: FP32 master parameters, BF16 copies, the
    feature frequencies and the ``lcs_mlp_t`` describing them."""

    def __init__(self, params, freq, in_shift, in_scale, out_scale, device="cuda"):
        torch = _torch()
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(device).contiguous()
        self.freq = torch.as_tensor(np.asarray(freq, dtype=np.float32)).to(device).contiguous()
        if self.params.numel() != LCS_MLP_PARAMS or tuple(self.freq.shape) != (LCS_MLP_FREQ, 4):
            raise ValueError("parameter vector or frequency matrix has the wrong size")
        self.bf16 = torch.empty(LCS_MLP_BF16, dtype=torch.int16, device=device)
        d = lcs_mlp_t()
        d.freq = self.freq.data_ptr()
        for a in range(4):
            d.in_shift[a] = float(in_shift[a])
            d.in_scale[a] = float(in_scale[a])
        d.out_scale = float(out_scale)
        d.reserved = 0
        d.params = self.params.data_ptr()
        d.params_bf16 = self.bf16.data_ptr()
        self.desc = d
        self.refresh()

    @property
    def ref(self):
        return C.byref(self.desc)

    def refresh(self, stream=None):
        lcs_mlp_refresh_bf16(self.params, self.bf16, stream=stream)


def lcs_mlp_workspace_bytes(batch: int, training: bool) -> int:
    return int(_lib.lcs_mlp_workspace_bytes(int(batch), 1 if training else 0))


def lcs_mlp_backward_scratch_bytes(batch: int) -> int:
    return int(_lib.lcs_mlp_backward_scratch_bytes(int(batch)))


def lcs_mlp_refresh_bf16(params, params_bf16, stream=None):
    _check(_lib.lcs_mlp_refresh_bf16(_ptr(params), _ptr(params_bf16), _stream_handle(stream)))


def _bytes_buffer(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 16), dtype=torch.uint8, device=device)


def lcs_mlp_forward(mlp: Mlp, xt, dx=None, workspace=None, training=False, stream=None):
    """dx [3, B] f32 for inputs xt [4, B] f32 (rows x, y, z, t)."""
    torch = _torch()
    B = int(xt.shape[1])
    dev = xt.device
    _need(xt, torch.float32, (4, B), "xt")
    if dx is None:
        dx = torch.empty((3, B), dtype=torch.float32, device=dev)
    _need(dx, torch.float32, (3, B), "dx")
    need = lcs_mlp_workspace_bytes(B, training)
    if workspace is None:
        workspace = _bytes_buffer(need, dev)
    _check(_lib.lcs_mlp_forward(mlp.ref, _ptr(xt), B, _ptr(dx), _ptr(workspace),
                                int(workspace.numel() * workspace.element_size()),
                                1 if training else 0, _stream_handle(stream)))
    return dx, workspace


def lcs_mlp_backward(mlp: Mlp, workspace, ddx, grads=None, scratch=None, stream=None):
    """Parameter gradient [LCS_MLP_PARAMS] f32 of sum(ddx * dx) for the batch
    whose training forward filled ``workspace``."""
    torch = _torch()
    B = int(ddx.shape[1])
    dev = ddx.device
    _need(ddx, torch.float32, (3, B), "ddx")
    if grads is None:
        grads = torch.empty(LCS_MLP_PARAMS, dtype=torch.float32, device=dev)
    _need(grads, torch.float32, (LCS_MLP_PARAMS,), "grads")
    if scratch is None:
        scratch = _bytes_buffer(lcs_mlp_backward_scratch_bytes(B), dev)
    _check(_lib.lcs_mlp_backward(mlp.ref, _ptr(workspace), _ptr(ddx), B, _ptr(grads), _ptr(scratch),
                                 int(scratch.numel() * scratch.element_size()),
                                 _stream_handle(stream)))
    return grads


def lcs_mse_grad(pred, target, grad=None, loss=None, want_grad=True, want_loss=True, stream=None):
    torch = _torch()
    n = int(pred.numel())
    if grad is None and want_grad:
        grad = torch.empty_like(pred)
    if loss is None and want_loss:
        loss = torch.empty(1, dtype=torch.float64, device=pred.device)
    _check(_lib.lcs_mse_grad(_ptr(pred), _ptr(target), n, _ptr(grad), _ptr(loss),
                             _stream_handle(stream)))
    return grad, loss


def lcs_adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                  stream=None):
    n = int(params.numel())
    _check(_lib.lcs_adam_step(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), n, float(lr),
                              float(beta1), float(beta2), float(eps), int(step),
                              _stream_handle(stream)))


def lcs_mlp_train_workspace_bytes(batch: int) -> int:
    return int(_lib.lcs_mlp_train_workspace_bytes(int(batch)))


def lcs_mlp_train(mlp: Mlp, xt, target, batch: int, first_step: int, n_steps: int,
                  total_steps: int, m, v, lr=2e-3, lr_final=1e-4, beta1=0.9, beta2=0.999,
                  eps=1e-8, losses=None, grads=None, workspace=None, stream=None):
    """n_steps fused Adam steps on consecutive batches of (xt [4, n], target [3, n]);
    returns (losses [n_steps] f64 or None, grads or None)."""
    torch = _torch()
    n = int(xt.shape[1])
    dev = xt.device
    _need(xt, torch.float32, (4, n), "xt")
    _need(target, torch.float32, (3, n), "target")
    for t, nm in ((m, "m"), (v, "v")):
        _need(t, torch.float32, (LCS_MLP_PARAMS,), nm)
    if losses is not None:
        _need(losses, torch.float64, (n_steps,), "losses")
    if grads is not None:
        _need(grads, torch.float32, (LCS_MLP_PARAMS,), "grads")
    if workspace is None:
        workspace = _bytes_buffer(lcs_mlp_train_workspace_bytes(batch), dev)
    _check(_lib.lcs_mlp_train(mlp.ref, _ptr(mlp.params), _ptr(mlp.bf16), _ptr(xt), _ptr(target), n,
                              int(batch), int(first_step), int(n_steps), int(total_steps),
                              float(lr), float(lr_final), float(beta1), float(beta2), float(eps),
                              _ptr(m), _ptr(v), _ptr(losses), _ptr(grads), _ptr(workspace),
                              int(workspace.numel() * workspace.element_size()),
                              _stream_handle(stream)))
    return losses, grads


def lcs_check_tile_count(seeds) -> int:
    sd = seed_grid_desc(seeds)
    return int(_lib.lcs_check_tile_count(C.byref(sd)))


def lcs_surrogate_compose(mlp: Mlp, seeds, t0: float, tau: float, n_windows: int, xf=None,
                          stream=None):
    """Surrogate flow map of the seed grid: n_windows composed windows of tau."""
    torch = _torch()
    dev = mlp.params.device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    if xf is None:
        xf = torch.empty((3, ns), dtype=torch.float32, device=dev)
    _need(xf, torch.float32, (3, ns), "xf")
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_surrogate_compose(mlp.ref, C.byref(sd), float(t0), float(tau), int(n_windows),
                                      _ptr(xf), _stream_handle(stream)))
    return xf


def lcs_surrogate_check(frames: DeviceFrames, seeds, t0: float, T: float, dt: float, xf, tol: float,
                        tile_err=None, tile_fail=None, n_fail=None, stream=None):
    """Per-tile check-sample error of a surrogate flow map and the failing tiles."""
    torch = _torch()
    dev = xf.device
    nt = lcs_check_tile_count(seeds)
    if tile_err is None:
        tile_err = torch.empty(nt, dtype=torch.float32, device=dev)
    if tile_fail is None:
        tile_fail = torch.empty(nt, dtype=torch.uint8, device=dev)
    if n_fail is None:
        n_fail = torch.empty(1, dtype=torch.int32, device=dev)
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    _need(xf, torch.float32, (3, ns), "xf")
    _need(tile_err, torch.float32, (nt,), "tile_err")
    _need(tile_fail, torch.uint8, (nt,), "tile_fail")
    _need(n_fail, torch.int32, (1,), "n_fail")
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_surrogate_check(frames.ref, C.byref(sd), float(t0), float(T), float(dt),
                                    _ptr(xf), float(tol), _ptr(tile_err), _ptr(tile_fail),
                                    _ptr(n_fail), _stream_handle(stream)))
    return tile_err, tile_fail, n_fail


def lcs_advect_tiles(frames: DeviceFrames, seeds, t0: float, T: float, dt: float, tile_fail, xf,
                     cell=None, flags=None, stream=None):
    torch = _torch()
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    _need(xf, torch.float32, (3, ns), "xf")
    _need(cell, torch.int64, (ns,), "cell")
    _need(flags, torch.uint8, (ns,), "flags")
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_advect_tiles(frames.ref, C.byref(sd), float(t0), float(T), float(dt),
                                 _ptr(tile_fail), _ptr(xf), _ptr(cell), _ptr(flags),
                                 _stream_handle(stream)))
    return xf


def lcs_surrogate_flowmap_workspace_bytes(frames: DeviceFrames, seeds,
                                          whole_grid_fraction: float = 0.25) -> int:
    sd = seed_grid_desc(seeds)
    return int(_lib.lcs_surrogate_flowmap_workspace_bytes(frames.ref, C.byref(sd),
                                                          float(whole_grid_fraction)))


def lcs_surrogate_flowmap(mlp: Mlp, frames: DeviceFrames, seeds, t0: float, tau: float,
                          n_windows: int, tol: float, dt: float, whole_grid_fraction: float = 0.25,
                          xf=None, flags=None, tile_err=None, want_flags=True, workspace=None,
                          stream=None):
    """Composed surrogate flow map with RK4 check samples and RK4 fallback of
    failing tiles (or of the whole grid), all inside the library.  Returns
    (xf, flags, n_fallback_tiles, whole_grid, tile_err)."""
    torch = _torch()
    dev = mlp.params.device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    nt = lcs_check_tile_count(seeds)
    if xf is None:
        xf = torch.empty((3, ns), dtype=torch.float32, device=dev)
    if flags is None and want_flags:
        flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    if tile_err is None:
        tile_err = torch.empty(nt, dtype=torch.float32, device=dev)
    _need(xf, torch.float32, (3, ns), "xf")
    _need(flags, torch.uint8, (ns,), "flags")
    _need(tile_err, torch.float32, (nt,), "tile_err")
    if workspace is None:
        workspace = _bytes_buffer(
            lcs_surrogate_flowmap_workspace_bytes(frames, seeds, whole_grid_fraction), dev)
    nf, whole = C.c_int32(), C.c_int32()
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_surrogate_flowmap(mlp.ref, frames.ref, C.byref(sd), float(t0), float(tau),
                                      int(n_windows), float(tol), float(dt),
                                      float(whole_grid_fraction), _ptr(xf), _ptr(flags),
                                      _ptr(tile_err), C.byref(nf), C.byref(whole), _ptr(workspace),
                                      int(workspace.numel() * workspace.element_size()),
                                      _stream_handle(stream)))
    return xf, flags, int(nf.value), bool(whole.value), tile_err


def lcs_sub(a, b, out=None, stream=None):
    torch = _torch()
    if out is None:
        out = torch.empty_like(a)
    _need(a, torch.float32, tuple(a.shape), "a")
    _need(b, torch.float32, tuple(a.shape), "b")
    _need(out, torch.float32, tuple(a.shape), "out")
    _check(_lib.lcs_sub(_ptr(a), _ptr(b), int(a.numel()), _ptr(out), _stream_handle(stream)))
    return out


# ---------------------------------------------------------------------------
# Unstructured meshes
# ---------------------------------------------------------------------------

LCS_FLAG_LOST = 16


class lcs_mesh_desc_t(C.Structure):
    _fields_ = [("dim", C.c_int32), ("reserved", C.c_int32), ("n_nodes", C.c_int64),
                ("n_cells", C.c_int64), ("nodes", C.c_void_p), ("cells", C.c_void_p)]


class lcs_mesh_info_t(C.Structure):
    _fields_ = [("dim", C.c_int32), ("reserved", C.c_int32), ("n_nodes", C.c_int64),
                ("n_cells", C.c_int64), ("n_boundary_faces", C.c_int64),
                ("buckets", C.c_int64 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("device_bytes", C.c_int64)]


class lcs_mesh_frames_t(C.Structure):
    _fields_ = [("n_frames", C.c_int32), ("reserved", C.c_int32), ("t_first", C.c_double),
                ("dt_frame", C.c_double), ("u", C.c_void_p)]


class Mesh:
    """Device mesh object (lcs_mesh_create) built from a host mesh with
    ``dim``, ``nodes`` (n_nodes x dim) and ``cells`` (n_cells x dim+1)."""

    def __init__(self, mesh, device="cuda", stream=None):
        torch = _torch()
        self.dim = int(mesh.dim)
        nodes = torch.from_numpy(np.ascontiguousarray(mesh.nodes, dtype=np.float64)).to(device)
        cells = torch.from_numpy(np.ascontiguousarray(mesh.cells, dtype=np.int32)).to(device)
        d = lcs_mesh_desc_t()
        d.dim = self.dim
        d.reserved = 0
        d.n_nodes = int(nodes.shape[0])
        d.n_cells = int(cells.shape[0])
        d.nodes = nodes.data_ptr()
        d.cells = cells.data_ptr()
        self.n_nodes = int(d.n_nodes)
        self.n_cells = int(d.n_cells)
        self.device = nodes.device
        h = C.c_void_p()
        _check(_lib.lcs_mesh_create(C.byref(d), C.byref(h), _stream_handle(stream)))
        self.h = h

    def info(self) -> dict:
        i = lcs_mesh_info_t()
        _check(_lib.lcs_mesh_info(self.h, C.byref(i)))
        return dict(dim=i.dim, n_nodes=i.n_nodes, n_cells=i.n_cells,
                    n_boundary_faces=i.n_boundary_faces, buckets=list(i.buckets),
                    lo=list(i.lo), hi=list(i.hi), device_bytes=i.device_bytes)

    def close(self):
        if getattr(self, "h", None):
            _lib.lcs_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MeshFrames:
    """Nodal velocity frames of a mesh in the layout lcs_mesh_frames_t reads:
    [n_frames][n_nodes][S] FP32, S = 4 in 3D (one unused value), 2 in 2D."""

    def __init__(self, mf, device="cuda", tensor=None):
        torch = _torch()
        dim = mf.mesh.dim
        S = 4 if dim == 3 else 2
        if tensor is None:
            a = np.zeros((mf.n_frames, mf.mesh.n_nodes, S), dtype=np.float32)
            a[..., :dim] = mf.u
            tensor = torch.from_numpy(a).to(device)
        _need(tensor, torch.float32, (mf.n_frames, mf.mesh.n_nodes, S), "mesh frames")
        self.u = tensor
        self.mf = mf
        d = lcs_mesh_frames_t()
        d.n_frames = int(mf.n_frames)
        d.reserved = 0
        d.t_first = float(mf.t_first)
        d.dt_frame = float(mf.dt_frame)
        d.u = tensor.data_ptr()
        self.desc = d

    @property
    def ref(self):
        return C.byref(self.desc)


def lcs_mesh_locate(mesh: Mesh, x, cell=None, lam=None, want_lam=True, stream=None):
    """Cell (int64; -1 outside, -2 search limit) and barycentric coordinates of points x (dim x n)."""
    torch = _torch()
    d, n = mesh.dim, int(x.shape[1])
    _need(x, torch.float32, (d, n), "x")
    if cell is None:
        cell = torch.empty(n, dtype=torch.int64, device=x.device)
    if lam is None and want_lam:
        lam = torch.empty((d + 1, n), dtype=torch.float32, device=x.device)
    _need(cell, torch.int64, (n,), "cell")
    _need(lam, torch.float32, (d + 1, n), "lam")
    _check(_lib.lcs_mesh_locate(mesh.h, _ptr(x), n, _ptr(cell), _ptr(lam), _stream_handle(stream)))
    return cell, lam


def lcs_mesh_velocity_at(mesh: Mesh, frames: MeshFrames, x, t, u=None, cell=None, stream=None):
    """u(x, t) on the mesh (NaN outside) and the cell of every point."""
    torch = _torch()
    d, n = mesh.dim, int(x.shape[1])
    _need(x, torch.float32, (d, n), "x")
    if not isinstance(t, torch.Tensor):
        t = torch.full((n,), float(t), dtype=torch.float64, device=x.device)
    _need(t, torch.float64, (n,), "t")
    if u is None:
        u = torch.empty((d, n), dtype=torch.float32, device=x.device)
    if cell is None:
        cell = torch.empty(n, dtype=torch.int64, device=x.device)
    _need(u, torch.float32, (d, n), "u")
    _need(cell, torch.int64, (n,), "cell")
    _check(_lib.lcs_mesh_velocity_at(mesh.h, frames.ref, _ptr(x), _ptr(t), n, _ptr(u), _ptr(cell),
                                     _stream_handle(stream)))
    return u, cell


def lcs_mesh_advect(mesh: Mesh, frames: MeshFrames, seeds, t0: float, T: float, dt: float,
                    xf=None, cell=None, flags=None, want_cell=True, want_flags=True, stream=None):
    """Flow map of a (non-periodic) seed grid through mesh velocity frames."""
    torch = _torch()
    dev = frames.u.device
    d = mesh.dim
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    if xf is None:
        xf = torch.empty((d, ns), dtype=torch.float32, device=dev)
    if cell is None and want_cell:
        cell = torch.empty(ns, dtype=torch.int64, device=dev)
    if flags is None and want_flags:
        flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    _need(xf, torch.float32, (d, ns), "xf")
    _need(cell, torch.int64, (ns,), "cell")
    _need(flags, torch.uint8, (ns,), "flags")
    sd = seed_grid_desc(seeds)
    _check(_lib.lcs_mesh_advect(mesh.h, frames.ref, C.byref(sd), float(t0), float(T), float(dt),
                                _ptr(xf), _ptr(cell), _ptr(flags), _stream_handle(stream)))
    return xf, cell, flags


def lcs_mesh_advect_points(mesh: Mesh, frames: MeshFrames, x0, t0, T: float, dt: float, xf=None,
                           cell=None, flags=None, want_cell=True, want_flags=True, stream=None):
    """Flow map of points x0 (dim x n, FP32) with start times t0 (FP64) on the mesh."""
    torch = _torch()
    d, n = mesh.dim, int(x0.shape[1])
    dev = x0.device
    if not isinstance(t0, torch.Tensor):
        t0 = torch.full((n,), float(t0), dtype=torch.float64, device=dev)
    if xf is None:
        xf = torch.empty((d, n), dtype=torch.float32, device=dev)
    if cell is None and want_cell:
        cell = torch.empty(n, dtype=torch.int64, device=dev)
    if flags is None and want_flags:
        flags = torch.empty(n, dtype=torch.uint8, device=dev)
    _need(x0, torch.float32, (d, n), "x0")
    _need(t0, torch.float64, (n,), "t0")
    _need(xf, torch.float32, (d, n), "xf")
    _need(cell, torch.int64, (n,), "cell")
    _need(flags, torch.uint8, (n,), "flags")
    _check(_lib.lcs_mesh_advect_points(mesh.h, frames.ref, _ptr(x0), _ptr(t0), n, float(T),
                                       float(dt), _ptr(xf), _ptr(cell), _ptr(flags),
                                       _stream_handle(stream)))
    return xf, cell, flags
