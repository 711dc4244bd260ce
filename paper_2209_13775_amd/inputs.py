"""Seeded synthetic inputs: velocity frames, seed grids and t0 windows.

This module produces *inputs* only.  It holds none of the flow-map method's
arithmetic (no interpolation, no integration, no differencing, no
eigen-analysis); both the HIP path and the FP64 oracle consume what it
returns.

Layout of every frame set: one array per velocity component, shaped
``(F, n2, n1, n0)`` in 3D or ``(F, n1, n0)`` in 2D, axis 0 (x, index i)
fastest in memory.  Node ``i`` of a non-periodic axis sits at
``origin + i*h`` with ``h = extent/(n-1)``; a periodic axis of period ``L``
holds ``n`` nodes at ``i*L/n`` (no duplicated end point).  Frame ``f`` is the
field at ``t_first + f*dt_frame``.

Fields
------
* double gyre (the standard 2D test case of Shadden, Lekien & Marsden 2005,
  named as the 2D Cartesian application in Sec. 3.2 of the paper);
* time-dependent ABC flow (3D, periodic);
* divergence-free random-Fourier field (3D, periodic, Kolmogorov spectrum,
  Ornstein-Uhlenbeck time correlation);
* small analytic test fields (linear saddle, uniform stream, multilinear
  polynomial fields) used to pin the oracle.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# Descriptors (plain data; no arithmetic of the method)
# ---------------------------------------------------------------------------


@dataclass
class FrameSet:
    """Gridded, time-dependent velocity data in memory (NumPy, host)."""

    dim: int
    n: Tuple[int, int, int]            # nodes per axis, n[2] == 1 in 2D
    origin: Tuple[float, float, float]
    spacing: Tuple[float, float, float]
    periodic: Tuple[bool, bool, bool]
    t_first: float
    dt_frame: float
    u: List[np.ndarray]                # dim arrays, (F, n2, n1, n0) or (F, n1, n0)

    @property
    def n_frames(self) -> int:
        return int(self.u[0].shape[0])

    @property
    def periodic_mask(self) -> int:
        return sum((1 << a) for a in range(3) if self.periodic[a])

    def astype(self, dtype) -> "FrameSet":
        return FrameSet(self.dim, self.n, self.origin, self.spacing, self.periodic,
                        self.t_first, self.dt_frame,
                        [np.ascontiguousarray(c, dtype=dtype) for c in self.u])

    def extent(self, a: int) -> float:
        """Length of axis ``a``: the period if periodic, else max-min."""
        if self.periodic[a]:
            return self.n[a] * self.spacing[a]
        return (self.n[a] - 1) * self.spacing[a]


@dataclass
class SeedGrid:
    """Structured seed grid: seed (i,j,k) sits at origin + (i,j,k)*spacing."""

    dim: int
    n: Tuple[int, int, int]
    origin: Tuple[float, float, float]
    spacing: Tuple[float, float, float]
    periodic: Tuple[bool, bool, bool] = (False, False, False)

    @property
    def count(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def periodic_mask(self) -> int:
        return sum((1 << a) for a in range(3) if self.periodic[a])

    def index_of(self, ijk: np.ndarray) -> np.ndarray:
        """Linear (x fastest) index of integer seed coordinates, shape (dim, m)."""
        ijk = np.asarray(ijk, dtype=np.int64)
        idx = ijk[0].copy()
        if self.dim >= 2:
            idx += self.n[0] * ijk[1]
        if self.dim == 3:
            idx += self.n[0] * self.n[1] * ijk[2]
        return idx

    def coords_of(self, idx: np.ndarray) -> np.ndarray:
        idx = np.asarray(idx, dtype=np.int64)
        i = idx % self.n[0]
        r = idx // self.n[0]
        if self.dim == 2:
            return np.stack([i, r])
        j = r % self.n[1]
        k = r // self.n[1]
        return np.stack([i, j, k])


def linspace_seeds(dim, n, lo, hi) -> SeedGrid:
    """Node-inclusive seed grid on [lo, hi] per axis (non-periodic)."""
    n3 = tuple(list(n) + [1] * (3 - len(n)))
    lo3 = tuple(list(lo) + [0.0] * (3 - len(lo)))
    sp = tuple((hi[a] - lo[a]) / (n[a] - 1) if a < dim else 1.0 for a in range(3))
    return SeedGrid(dim, n3, lo3, sp, (False, False, False))


def periodic_seeds(dim, n, period) -> SeedGrid:
    """Seeds at i*L/n on every (periodic) axis."""
    n3 = tuple(list(n) + [1] * (3 - len(n)))
    sp = tuple(period[a] / n[a] if a < dim else 1.0 for a in range(3))
    per = tuple(a < dim for a in range(3))
    return SeedGrid(dim, n3, (0.0, 0.0, 0.0), sp, per)


# ---------------------------------------------------------------------------
# Sampling helpers
# ---------------------------------------------------------------------------


def _node_axes(n, origin, spacing, dim):
    return [origin[a] + np.arange(n[a], dtype=np.float64) * spacing[a] for a in range(dim)]


def sample_field(fn: Callable, dim: int, n, origin, spacing, periodic, t_first, dt_frame,
                 n_frames: int, dtype=np.float64) -> FrameSet:
    """Sample an analytic field ``fn(x, y[, z], t) -> tuple of components`` on nodes.

    ``fn`` receives broadcastable FP64 coordinate arrays (x varies along the
    last axis) and must return ``dim`` arrays broadcastable to the node grid.
    """
    n3 = tuple(list(n) + [1] * (3 - len(n)))
    o3 = tuple(list(origin) + [0.0] * (3 - len(origin)))
    s3 = tuple(list(spacing) + [1.0] * (3 - len(spacing)))
    p3 = tuple(list(periodic) + [False] * (3 - len(periodic)))
    ax = _node_axes(n3, o3, s3, dim)
    shape = tuple(n3[a] for a in reversed(range(dim)))
    comps = [np.empty((n_frames,) + shape, dtype=dtype) for _ in range(dim)]
    if dim == 2:
        X = ax[0][None, :]
        Y = ax[1][:, None]
        coords = (X, Y)
    else:
        X = ax[0][None, None, :]
        Y = ax[1][None, :, None]
        Z = ax[2][:, None, None]
        coords = (X, Y, Z)
    for f in range(n_frames):
        t = t_first + f * dt_frame
        vals = fn(*coords, t)
        for c in range(dim):
            comps[c][f] = np.broadcast_to(vals[c], shape)
    return FrameSet(dim, n3, o3, s3, p3, float(t_first), float(dt_frame), comps)


# ---------------------------------------------------------------------------
# Double gyre (Shadden, Lekien & Marsden 2005), 2D Cartesian application
# ---------------------------------------------------------------------------


def double_gyre_velocity(x, y, t, A=0.1, eps=0.25, omega=2 * math.pi / 10):
    """Analytic double-gyre velocity (stream function A sin(pi f) sin(pi y))."""
    a = eps * np.sin(omega * t)
    b = 1.0 - 2.0 * eps * np.sin(omega * t)
    f = a * x * x + b * x
    dfdx = 2.0 * a * x + b
    u = -math.pi * A * np.sin(math.pi * f) * np.cos(math.pi * y)
    v = math.pi * A * np.cos(math.pi * f) * np.sin(math.pi * y) * dfdx
    return u, v


def double_gyre_frames(nx=201, ny=101, n_frames=21, dt_frame=1.0, t_first=0.0,
                       A=0.1, eps=0.25, omega=2 * math.pi / 10, dtype=np.float64) -> FrameSet:
    """Double gyre on [0,2]x[0,1], nx x ny nodes (node-inclusive)."""
    hx = 2.0 / (nx - 1)
    hy = 1.0 / (ny - 1)
    return sample_field(lambda X, Y, t: double_gyre_velocity(X, Y, t, A, eps, omega),
                        2, (nx, ny), (0.0, 0.0), (hx, hy), (False, False),
                        t_first, dt_frame, n_frames, dtype)


# ---------------------------------------------------------------------------
# Time-dependent ABC flow, 3D periodic on [0, 2pi)^3
# ---------------------------------------------------------------------------

ABC_B = math.sqrt(2.0)
ABC_C = 1.0


def abc_A(t):
    """A(t) = sqrt(3) + 0.1 sin(2 pi t / 10) (additive reading of the modulation)."""
    return math.sqrt(3.0) + 0.1 * math.sin(2.0 * math.pi * t / 10.0)


def abc_velocity(x, y, z, t):
    A = abc_A(t)
    u = A * np.sin(z) + ABC_C * np.cos(y)
    v = ABC_B * np.sin(x) + A * np.cos(z)
    w = ABC_C * np.sin(y) + ABC_B * np.cos(x)
    return u, v, w


def abc_frames(n=128, n_frames=33, dt_frame=0.5, t_first=0.0, dtype=np.float32) -> FrameSet:
    """ABC flow sampled in FP64 on an n^3 periodic grid, stored as ``dtype``."""
    L = 2.0 * math.pi
    h = L / n
    ax = np.arange(n, dtype=np.float64) * h
    sx, cx = np.sin(ax), np.cos(ax)
    comps = [np.empty((n_frames, n, n, n), dtype=dtype) for _ in range(3)]
    for f in range(n_frames):
        A = abc_A(t_first + f * dt_frame)
        # u depends on (y, z), v on (x, z), w on (x, y); x is the last (fastest) axis
        comps[0][f] = np.broadcast_to(A * sx[:, None, None] + ABC_C * cx[None, :, None], (n, n, n))
        comps[1][f] = np.broadcast_to(ABC_B * sx[None, None, :] + A * cx[:, None, None], (n, n, n))
        comps[2][f] = np.broadcast_to(ABC_C * sx[None, :, None] + ABC_B * cx[None, None, :], (n, n, n))
    return FrameSet(3, (n, n, n), (0.0, 0.0, 0.0), (h, h, h), (True, True, True),
                    float(t_first), float(dt_frame), comps)


# ---------------------------------------------------------------------------
# Small analytic fields used to pin the oracle
# ---------------------------------------------------------------------------


def saddle_frames(lam=0.5, n=13, half=3.0, n_frames=2, t_first=0.0, dt_frame=10.0,
                  dim=2, lam_rate=0.0) -> FrameSet:
    """Linear saddle u = lam(t)*(x, -y[, 0]) on [-half, half]^dim.

    ``lam(t) = lam + lam_rate*t`` is linear in time, so bilinear-in-space and
    linear-in-time interpolation reproduce it exactly.
    """
    h = 2.0 * half / (n - 1)
    if dim == 2:
        fn = lambda X, Y, t: ((lam + lam_rate * t) * X, -(lam + lam_rate * t) * Y)
        return sample_field(fn, 2, (n, n), (-half, -half), (h, h), (False, False),
                            t_first, dt_frame, n_frames)
    fn = lambda X, Y, Z, t: ((lam + lam_rate * t) * X, -(lam + lam_rate * t) * Y, 0.0 * Z)
    return sample_field(fn, 3, (n, n, n), (-half,) * 3, (h,) * 3, (False,) * 3,
                        t_first, dt_frame, n_frames)


def uniform_frames(c, dim=2, n=9, lo=0.0, hi=1.0, n_frames=2, t_first=0.0, dt_frame=10.0,
                   periodic=False) -> FrameSet:
    """Uniform stream u = c on a box (closed, or periodic with period hi-lo)."""
    if periodic:
        h = (hi - lo) / n
    else:
        h = (hi - lo) / (n - 1)
    nn = (n,) * dim
    if dim == 2:
        fn = lambda X, Y, t: (c[0] + 0 * X, c[1] + 0 * Y)
    else:
        fn = lambda X, Y, Z, t: (c[0] + 0 * X, c[1] + 0 * Y, c[2] + 0 * Z)
    return sample_field(fn, dim, nn, (lo,) * dim, (h,) * dim, (periodic,) * dim,
                        t_first, dt_frame, n_frames)


def bilinear_rotor_frames(n=17, half=2.0, n_frames=3, dt_frame=5.0, t_first=0.0) -> FrameSet:
    """A nonlinear but bilinear-in-space, linear-in-time 2D field.

    u = (-y + 0.3 x y) (1 + 0.05 t),  v = (x - 0.2 x y) (1 + 0.05 t).
    Bilinear-in-space / linear-in-time interpolation reproduces it exactly, so
    gridded integration equals integration of the analytic polynomial field.
    """
    h = 2.0 * half / (n - 1)

    def fn(X, Y, t):
        s = 1.0 + 0.05 * t
        return ((-Y + 0.3 * X * Y) * s, (X - 0.2 * X * Y) * s)

    return sample_field(fn, 2, (n, n), (-half, -half), (h, h), (False, False),
                        t_first, dt_frame, n_frames)


def bilinear_rotor_rhs(t, z):
    x, y = z
    s = 1.0 + 0.05 * t
    return [(-y + 0.3 * x * y) * s, (x - 0.2 * x * y) * s]


def random_frames(dim, n, n_frames, seed, periodic=None, origin=None, spacing=None,
                  t_first=0.0, dt_frame=1.0) -> FrameSet:
    """Frames of i.i.d. normal values (for interpolation brute-force tests)."""
    rng = np.random.default_rng(seed)
    n3 = tuple(list(n) + [1] * (3 - len(n)))
    periodic = tuple(periodic) if periodic is not None else (False,) * dim
    p3 = tuple(list(periodic) + [False] * (3 - dim))
    o3 = tuple(list(origin) if origin is not None else [0.0] * dim) + (0.0,) * (3 - dim)
    s3 = tuple(list(spacing) if spacing is not None else [1.0] * dim) + (1.0,) * (3 - dim)
    shape = (n_frames,) + tuple(n3[a] for a in reversed(range(dim)))
    comps = [rng.standard_normal(shape) for _ in range(dim)]
    return FrameSet(dim, n3, o3, s3, p3, float(t_first), float(dt_frame), comps)


# ---------------------------------------------------------------------------
# Divergence-free random-Fourier field (3D periodic)
# ---------------------------------------------------------------------------


def random_fourier_frames(n=256, n_frames=65, dt_frame=0.125, kmax=32, tau=2.0, seed=1,
                          t_first=0.0, device=None) -> FrameSet:
    """Divergence-free random-Fourier velocity field on [0, 2pi)^3, FP32 frames.

    Recipe: integer wavevectors with 1 <= |k| <= kmax (half spectrum of a real
    FFT); each mode amplitude is P(k) xi_k(t) s(|k|) with the solenoidal
    projector P = I - k k^T/|k|^2 and s^2 = E(k)/(4 pi k^2), E(k) ~ k^(-5/3);
    xi_k is a complex Gaussian Ornstein-Uhlenbeck process with correlation
    exp(-|dt|/tau), stationary at t = 0 (random phases).  An inverse real FFT
    gives the nodes; one global constant then makes the RMS speed over all
    frames 1.  The draws come from numpy.random.default_rng(seed), mode by mode
    in a fixed order, so every device produces the same field.

    ``device`` (a torch device) runs the inverse FFTs there and returns the
    frames as device tensors in ``u`` (large grids); otherwise NumPy arrays.
    """
    rng = np.random.default_rng(seed)
    kk = np.fft.fftfreq(n, d=1.0 / n)
    kr = np.fft.rfftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(kk, kk, kr, indexing="ij")
    K2 = KX * KX + KY * KY + KZ * KZ
    mask = (K2 >= 1.0) & (K2 <= kmax * kmax)
    pos = np.flatnonzero(mask.ravel())
    kx, ky, kz = KX.ravel()[pos], KY.ravel()[pos], KZ.ravel()[pos]
    kmag = np.sqrt(K2.ravel()[pos])
    amp = np.sqrt(kmag ** (-5.0 / 3.0) / (4.0 * math.pi * kmag * kmag))
    khat = np.stack([kx, ky, kz]) / kmag
    m = pos.size
    rho = math.exp(-dt_frame / tau)
    innov = math.sqrt(1.0 - rho * rho)

    def draw():
        return (rng.standard_normal((3, m)) + 1j * rng.standard_normal((3, m))) / math.sqrt(2.0)

    spec_shape = (n, n, n // 2 + 1)
    torch = None
    if device is not None:
        import torch  # noqa: F811  (plumbing: FFTs and storage on the GPU)
        pos_t = torch.from_numpy(pos).to(device)
    xi = draw()
    comps = []
    sumsq = 0.0
    if torch is not None:
        u_dev = [torch.empty((n_frames, n, n, n), dtype=torch.float32, device=device)
                 for _ in range(3)]
    for f in range(n_frames):
        if f > 0:
            xi = rho * xi + innov * draw()
        a = xi * amp[None]
        a = a - khat * (khat * a).sum(axis=0)[None]          # solenoidal projection
        frame = []
        for c in range(3):
            if torch is None:
                spec = np.zeros(np.prod(spec_shape), dtype=np.complex128)
                spec[pos] = a[c]
                real = np.fft.irfftn(spec.reshape(spec_shape), s=(n, n, n), axes=(0, 1, 2))
                real = (real * n ** 3).astype(np.float32)
                sumsq += float(np.sum(real.astype(np.float64) ** 2))
            else:
                spec = torch.zeros(int(np.prod(spec_shape)), dtype=torch.complex128, device=device)
                spec[pos_t] = torch.from_numpy(a[c]).to(device)
                real = torch.fft.irfftn(spec.reshape(spec_shape), s=(n, n, n), dim=(0, 1, 2))
                u_dev[c][f] = (real * float(n ** 3)).to(torch.float32)
                sumsq += float((u_dev[c][f].double() ** 2).sum().item())
                del spec, real
                real = None
            frame.append(real)
        comps.append(frame)
    rms = math.sqrt(sumsq / (n_frames * n ** 3 * 1.0))
    scale = 1.0 / rms
    if torch is None:
        u = [np.stack([comps[f][c] for f in range(n_frames)]) for c in range(3)]
        for c in range(3):
            u[c] *= np.float32(scale)
    else:
        u = u_dev
        for c in range(3):
            u[c].mul_(scale)
    h = 2.0 * math.pi / n
    return FrameSet(3, (n, n, n), (0.0, 0.0, 0.0), (h, h, h), (True, True, True),
                    float(t_first), float(dt_frame), u)


# ---------------------------------------------------------------------------
# Batched t0 windows
# ---------------------------------------------------------------------------


def t0_windows(n_windows=64, t0_range=(0.0, 10.0), T_choices=(5.0, 7.5, 10.0, 12.5, 15.0),
               seed=0) -> np.ndarray:
    """(t0, T) pairs: t0 uniform on t0_range first, then T from T_choices."""
    rng = np.random.default_rng(seed)
    t0 = rng.uniform(t0_range[0], t0_range[1], n_windows)
    T = rng.choice(np.asarray(T_choices, dtype=np.float64), n_windows)
    return np.stack([t0, T], axis=1)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

WORKLOADS = {
    "double_gyre_201x101_seeds256x128": dict(
        field="double_gyre", n=(201, 101), frames=21, dt_frame=1.0, seeds=(256, 128),
        t0=0.0, T=10.0, dt=0.05),
    "abc_128cubed_seeds256cubed": dict(
        field="abc", n=128, frames=33, dt_frame=0.5, seeds=(256, 256, 256),
        t0=0.0, T=8.0, dt=0.02),
    "double_gyre_batched_1025x513_64windows": dict(
        field="double_gyre", n=(1025, 513), frames=101, dt_frame=0.25, seeds=(1024, 512),
        windows=64, dt=0.05),
    "random_fourier_256cubed_seeds512x512x256": dict(
        field="random_fourier", n=256, frames=65, dt_frame=0.125, seeds=(512, 512, 256),
        t0=4.0, T=4.0, dt=0.01),
}


# ---------------------------------------------------------------------------
# 2D periodic test field (time-modulated Taylor-Green cells)
# ---------------------------------------------------------------------------


def taylor_green_frames(n=64, n_frames=9, dt_frame=0.5, t_first=0.0, amp=0.5) -> FrameSet:
    """u = amp (1 + 0.3 sin t) (sin x cos y, -cos x sin y) + (0.2, 0.1) on [0, 2pi)^2."""
    L = 2.0 * math.pi
    h = L / n

    def fn(X, Y, t):
        s = amp * (1.0 + 0.3 * math.sin(t))
        return (s * np.sin(X) * np.cos(Y) + 0.2, -s * np.cos(X) * np.sin(Y) + 0.1)

    return sample_field(fn, 2, (n, n), (0.0, 0.0), (h, h), (True, True), t_first, dt_frame,
                        n_frames)


# ---------------------------------------------------------------------------
# Unstructured meshes (triangles in 2D, tetrahedra in 3D) and nodal velocity
# ---------------------------------------------------------------------------
#
# The paper's unstructured applications (a coronary stenosis, 2D; an aortic
# aneurysm with about one million tetrahedra, 3D) are CFD data that is not
# available.  Synthetic meshes stand in for them: a box cut into cells of a
# lattice, every square split into two triangles along the same diagonal, every
# cube into the six tetrahedra that share its main diagonal (Kuhn's split, which
# is conforming across the lattice), with the interior nodes jittered so that
# no two cells have the same shape.  Boundary nodes move only along the
# boundary, so the union of the cells is exactly the box.


@dataclass
class Mesh:
    """Conforming triangle (dim 2) or tetrahedron (dim 3) mesh on the host."""

    dim: int
    nodes: np.ndarray   # (n_nodes, dim) FP64 coordinates
    cells: np.ndarray   # (n_cells, dim + 1) int32 node ids

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])


@dataclass
class MeshFrames:
    """Velocity at the nodes of a fixed mesh: u[f, node, c] is component c at
    node ``node`` in frame f, the field at t_first + f*dt_frame."""

    mesh: Mesh
    t_first: float
    dt_frame: float
    u: np.ndarray       # (F, n_nodes, dim)

    @property
    def dim(self) -> int:
        return self.mesh.dim

    @property
    def n_frames(self) -> int:
        return int(self.u.shape[0])


def _signed_measure(nodes: np.ndarray, cells: np.ndarray) -> np.ndarray:
    """Signed area (2D) or 6x signed volume (3D) of every cell (mesh checks)."""
    v = [nodes[cells[:, i]] for i in range(cells.shape[1])]
    e = [v[i] - v[0] for i in range(1, len(v))]
    if nodes.shape[1] == 2:
        return e[0][:, 0] * e[1][:, 1] - e[0][:, 1] * e[1][:, 0]
    return np.einsum("ij,ij->i", e[0], np.cross(e[1], e[2]))


def box_mesh(dim: int, cells_per_axis, lo, hi, jitter: float = 0.0, seed: int = 0,
             shuffle: bool = False) -> Mesh:
    """Lattice mesh of the box [lo, hi]: ``cells_per_axis`` squares or cubes per
    axis, split into 2 triangles or 6 tetrahedra each.  ``jitter`` moves each
    interior node coordinate by U(-jitter, jitter) lattice steps (boundary
    nodes move only along the boundary).  ``shuffle`` renumbers nodes and cells
    and permutes the vertex order inside each cell at random (the mesh is the
    same; only its numbering becomes unstructured)."""
    m = [int(c) for c in cells_per_axis][:dim]
    lo = [float(v) for v in lo][:dim]
    hi = [float(v) for v in hi][:dim]
    h = [(hi[a] - lo[a]) / m[a] for a in range(dim)]
    rng = np.random.default_rng(seed)
    ax = [np.arange(m[a] + 1) for a in range(dim)]
    grids = np.meshgrid(*ax, indexing="ij")            # axis 0 = x
    ijk = np.stack([g.transpose(tuple(reversed(range(dim)))).ravel() for g in grids], axis=1)
    nodes = np.stack([lo[a] + ijk[:, a] * h[a] for a in range(dim)], axis=1)
    if jitter > 0.0:
        d = rng.uniform(-jitter, jitter, size=nodes.shape)
        interior = (ijk > 0) & (ijk < np.array(m)[None, :])
        nodes = nodes + d * interior * np.array(h)[None, :]
        for a in range(dim):                           # keep the walls exact
            nodes[ijk[:, a] == 0, a] = lo[a]
            nodes[ijk[:, a] == m[a], a] = hi[a]

    def nid(i, j, k=0):
        return i + (m[0] + 1) * (j + (m[1] + 1) * k)

    if dim == 2:
        j, i = np.meshgrid(np.arange(m[1]), np.arange(m[0]), indexing="ij")
        i, j = i.ravel(), j.ravel()
        c00, c10, c01, c11 = nid(i, j), nid(i + 1, j), nid(i, j + 1), nid(i + 1, j + 1)
        tris = np.stack([np.stack([c00, c10, c11], 1), np.stack([c00, c11, c01], 1)], axis=1)
        cells = tris.reshape(-1, 3)
    else:
        k, j, i = np.meshgrid(np.arange(m[2]), np.arange(m[1]), np.arange(m[0]), indexing="ij")
        i, j, k = i.ravel(), j.ravel(), k.ravel()
        corner = [nid(i + (b & 1), j + ((b >> 1) & 1), k + ((b >> 2) & 1)) for b in range(8)]
        tets = []
        for perm in ((0, 1, 2), (1, 2, 0), (2, 0, 1), (0, 2, 1), (2, 1, 0), (1, 0, 2)):
            b1 = 1 << perm[0]
            b2 = b1 | (1 << perm[1])
            t = [corner[0], corner[b1], corner[b2], corner[7]]
            if perm in ((0, 2, 1), (2, 1, 0), (1, 0, 2)):      # odd: restore orientation
                t[1], t[2] = t[2], t[1]
            tets.append(np.stack(t, 1))
        cells = np.stack(tets, axis=1).reshape(-1, 4)
    cells = cells.astype(np.int32)
    meas = _signed_measure(nodes, cells)
    if not np.all(meas > 0):
        raise ValueError("jitter too large: a cell lost its orientation")
    if shuffle:
        pn = rng.permutation(nodes.shape[0])
        inv = np.empty_like(pn)
        inv[pn] = np.arange(pn.size)
        nodes = nodes[pn]
        cells = inv[cells].astype(np.int32)
        cells = cells[rng.permutation(cells.shape[0])]
        order = np.argsort(rng.random(cells.shape), axis=1)
        cells = np.take_along_axis(cells, order, axis=1).astype(np.int32)
    return Mesh(dim, np.ascontiguousarray(nodes), np.ascontiguousarray(cells))


def mesh_sample(fn: Callable, mesh: Mesh, n_frames: int, t_first: float, dt_frame: float,
                dtype=np.float64) -> MeshFrames:
    """Sample ``fn(x, y[, z], t) -> components`` at the mesh nodes in FP64."""
    u = np.empty((n_frames, mesh.n_nodes, mesh.dim), dtype=dtype)
    coords = [mesh.nodes[:, a] for a in range(mesh.dim)]
    for f in range(n_frames):
        vals = fn(*coords, t_first + f * dt_frame)
        for c in range(mesh.dim):
            u[f, :, c] = np.broadcast_to(vals[c], (mesh.n_nodes,))
    return MeshFrames(mesh, float(t_first), float(dt_frame), u)


def box_cells_velocity(x, y, z, t, eps=0.5, omega=2 * math.pi / 4):
    """Time-dependent cellular flow in the box [0, pi]^3: a Taylor-Green cell
    rolling about z plus eps sin(omega t) times the same cell rolling about x.
    Divergence-free, with no flow through any wall, chaotic mixing inside."""
    s = eps * np.sin(omega * t)
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z) + s * np.cos(x) * np.sin(y) * np.cos(z)
    w = -s * np.cos(x) * np.cos(y) * np.sin(z)
    return u, v, w


def double_gyre_mesh_frames(cells=(200, 100), n_frames=21, dt_frame=1.0, jitter=0.15, seed=0,
                            shuffle=False) -> MeshFrames:
    """Double gyre on a jittered triangle mesh of [0,2] x [0,1] (stands in for
    the 2D unstructured application)."""
    mesh = box_mesh(2, cells, (0.0, 0.0), (2.0, 1.0), jitter=jitter, seed=seed, shuffle=shuffle)
    return mesh_sample(double_gyre_velocity, mesh, n_frames, 0.0, dt_frame)


def box_cells_mesh_frames(cells=64, n_frames=41, dt_frame=0.25, jitter=0.15, seed=0,
                          shuffle=False) -> MeshFrames:
    """Cellular box flow on a jittered tetrahedron mesh of [0, pi]^3 (stands in
    for the 3D unstructured application)."""
    c = (cells,) * 3 if np.isscalar(cells) else tuple(cells)
    mesh = box_mesh(3, c, (0.0,) * 3, (math.pi,) * 3, jitter=jitter, seed=seed, shuffle=shuffle)
    return mesh_sample(box_cells_velocity, mesh, n_frames, 0.0, dt_frame)


WORKLOADS.update({
    "double_gyre_trimesh_200x100x2_seeds256x128": dict(
        field="double_gyre", mesh="tri", cells=(200, 100), frames=21, dt_frame=1.0,
        seeds=(256, 128), t0=0.0, T=10.0, dt=0.05),
    "box_cells_tetmesh_64cubed_x6_seeds192cubed": dict(
        field="box_cells", mesh="tet", cells=64, frames=41, dt_frame=0.25,
        seeds=(192, 192, 192), t0=0.0, T=8.0, dt=0.02),
})
