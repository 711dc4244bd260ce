"""Helpers shared by the GPU parity tests: run both sides, compare.

Parity bar (written in the tests that use these helpers):
* flow-map position: mean and p99 over tracers of |x_gpu - x_oracle| within
  1e-5 of the domain length (the paper's mean trajectory error e_S of
  Sec. 3.3, plus a tail quantile); the maximum is reported;
* FTLE: 1e-3 absolute on every seed whose stencil is clean on both sides;
* flags and cell index: bit-exact.  Cell index recomputed by the oracle from
  the GPU's own FP32 positions: every tracer.  Against the oracle's own run:
  every "unambiguous" tracer, i.e. one whose oracle run never brings a
  checked point within 1e-5 L of a wall (flags) and whose final position is
  not within 1e-5 L of a cell face (cell index).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

POS_TOL_FRAC = 1e-5
FTLE_TOL = 1e-3


def domain_length(fs) -> float:
    return max(fs.extent(a) for a in range(fs.dim))


@dataclass
class PosStats:
    mean: float
    p99: float
    max: float
    n: int
    n_over: int


def position_stats(x_gpu: np.ndarray, x_orc: np.ndarray, tol: float, mask=None) -> PosStats:
    err = np.linalg.norm(x_gpu.astype(np.float64) - x_orc, axis=0)
    if mask is not None:
        err = err[mask]
    if err.size == 0:
        return PosStats(0.0, 0.0, 0.0, 0, 0)
    return PosStats(float(err.mean()), float(np.quantile(err, 0.99)), float(err.max()),
                    int(err.size), int((err > tol).sum()))


def near_cell_face(fs, x: np.ndarray, tol: float) -> np.ndarray:
    """Positions within tol of a velocity-cell face along some axis."""
    near = np.zeros(x.shape[1], dtype=bool)
    for a in range(fs.dim):
        h = fs.spacing[a]
        s = (x[a] - fs.origin[a]) / h
        frac = s - np.floor(s)
        near |= (frac * h < tol) | ((1.0 - frac) * h < tol)
    return near


def assert_positions(st: PosStats, tol: float, what: str):
    msg = (f"{what}: e_S mean={st.mean:.3e} p99={st.p99:.3e} max={st.max:.3e} "
           f"(tol {tol:.1e}, {st.n_over}/{st.n} above)")
    print(msg)
    assert st.mean <= tol and st.p99 <= tol, msg


def neighbour_indices(g, idx: np.ndarray):
    """Seed indices of the -/+ neighbours along each axis (wrap or clamp)."""
    c = g.coords_of(idx)
    out_m, out_p = [], []
    for b in range(g.dim):
        n = g.n[b]
        cm = c.copy()
        cp = c.copy()
        if g.periodic[b]:
            cm[b] = (c[b] - 1) % n
            cp[b] = (c[b] + 1) % n
        else:
            cm[b] = np.maximum(c[b] - 1, 0)
            cp[b] = np.minimum(c[b] + 1, n - 1)
        out_m.append(g.index_of(cm))
        out_p.append(g.index_of(cp))
    return c, out_m, out_p


def sample_seeds(g, count: int, seed: int) -> np.ndarray:
    """A deterministic sample of seed indices, including the grid's corners."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(g.count, size=min(count, g.count), replace=False)
    corners = [0, g.n[0] - 1, g.count - 1, g.count - g.n[0]]
    return np.unique(np.concatenate([idx, np.array(corners, dtype=np.int64)]))


def oracle_sampled_ftle(orc, vel, g, idx, t0, T, dt):
    """Oracle flow map at the sampled seeds and their stencil neighbours, and
    the oracle FTLE at the sampled seeds (from its own positions)."""
    c, im, ip = neighbour_indices(g, idx)
    allidx = np.unique(np.concatenate([idx] + im + ip))
    xf, cell, flags, margin = orc.advect_seeds(vel, g, t0, T, dt, idx=allidx, margin=True)
    pos = {int(k): p for p, k in enumerate(allidx)}
    C = np.empty((g.dim * (g.dim + 1) // 2, idx.size))
    bad = np.zeros(idx.size, dtype=bool)
    for q, s in enumerate(idx):
        ps = pos[int(s)]
        xm = [xf[:, pos[int(im[b][q])]] for b in range(g.dim)]
        xp = [xf[:, pos[int(ip[b][q])]] for b in range(g.dim)]
        C[:, q] = orc.cg_point(g, c[:, q], xf[:, ps], xm, xp)
        used = [ps] + [pos[int(im[b][q])] for b in range(g.dim)] + [pos[int(ip[b][q])] for b in range(g.dim)]
        bad[q] = bool(np.any(flags[used]))
    lam, sig = orc.ftle(g.dim, C, T)
    sel = np.array([pos[int(s)] for s in idx])
    return dict(xf=xf[:, sel], cell=cell[sel], flags=flags[sel], margin=margin[sel],
                lam=lam, ftle=sig, stencil_bad=bad)


def oracle_sampled_ftle_mesh(mv, g, idx, t0, T, dt):
    """As oracle_sampled_ftle, for velocity on a mesh (oracle MeshVelocity)."""
    import oracle as orc
    c, im, ip = neighbour_indices(g, idx)
    allidx = np.unique(np.concatenate([idx] + im + ip))
    xf, cell, flags, margin, lam_margin = mv.advect_seeds(g, t0, T, dt, idx=allidx)
    pos = {int(k): p for p, k in enumerate(allidx)}
    C = np.empty((g.dim * (g.dim + 1) // 2, idx.size))
    bad = np.zeros(idx.size, dtype=bool)
    for q, s in enumerate(idx):
        ps = pos[int(s)]
        xm = [xf[:, pos[int(im[b][q])]] for b in range(g.dim)]
        xp = [xf[:, pos[int(ip[b][q])]] for b in range(g.dim)]
        C[:, q] = orc.cg_point(g, c[:, q], xf[:, ps], xm, xp)
        used = [ps] + [pos[int(im[b][q])] for b in range(g.dim)] + [pos[int(ip[b][q])] for b in range(g.dim)]
        bad[q] = bool(np.any(flags[used]))
    lam, sig = orc.ftle(g.dim, C, T)
    sel = np.array([pos[int(s)] for s in idx])
    return dict(xf=xf[:, sel], cell=cell[sel], flags=flags[sel], margin=margin[sel],
                lam_margin=lam_margin[sel], lam=lam, ftle=sig, stencil_bad=bad)


def mesh_barycentric(mesh, cell: np.ndarray, x: np.ndarray) -> np.ndarray:
    """FP64 barycentric coordinates (dim+1, m) of points x (dim, m) in the
    given cells of a host mesh, by a linear solve per point."""
    v = mesh.nodes[mesh.cells[cell]]                       # (m, dim+1, dim)
    E = np.transpose(v[:, 1:, :] - v[:, :1, :], (0, 2, 1))
    mu = np.linalg.solve(E, (x.T - v[:, 0, :])[..., None])[..., 0]
    return np.concatenate([1.0 - mu.sum(axis=1, keepdims=True), mu], axis=1).T
