"""Training and use of the learned flow-map surrogate (orchestration only).

Every arithmetic step runs in the HIP library through the C ABI: RK4 training
pairs (lcs_advect_points), displacements (lcs_sub), the training steps
(lcs_mlp_train: forward, loss gradient, backward, Adam), evaluation
(lcs_mlp_forward, lcs_mse_grad), composition over windows (lcs_surrogate_compose), check
samples and RK4 fallback (lcs_surrogate_flowmap) and the FTLE (lcs_cg_ftle).  torch provides device memory, random draws of the training
inputs and streams.

The surrogate predicts the displacement over a window tau of a point starting
at (x, t); the flow map over T = n_windows * tau is the composition
x_{k+1} = x_k + NN(x_k, t0 + k tau).  Tiles whose check samples (plain RK4)
differ by more than a tolerance are re-advected with plain RK4, which stays
the reference.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

from . import lcs

TWO_PI = 2.0 * math.pi


@dataclass
class SurrogateConfig:
    tau: float = 0.5
    n_windows: int = 8
    t0: float = 4.0
    dt: float = 0.01                 # RK4 step of training pairs, checks and fallback
    t0_choices: Sequence[float] = tuple(4.0 + 0.5 * k for k in range(8))
    period: float = TWO_PI
    sigma_x: float = 4.0             # spread of the integer spatial frequencies
    sigma_t: float = 1.0             # spread of the time frequencies
    speed_scale: float = 1.0         # RMS speed: out_scale = tau * speed_scale
    seed: int = 0


def make_frequencies(cfg: SurrogateConfig) -> np.ndarray:
    """B (64 x 4): integer spatial frequencies (exactly periodic features on the
    torus) and Gaussian time frequencies."""
    rng = np.random.default_rng(cfg.seed)
    bx = np.round(rng.standard_normal((lcs.LCS_MLP_FREQ, 3)) * cfg.sigma_x)
    bt = rng.standard_normal((lcs.LCS_MLP_FREQ, 1)) * cfg.sigma_t
    return np.concatenate([bx, bt], axis=1).astype(np.float32)


def init_params(seed: int) -> np.ndarray:
    """Uniform fan-in initialisation (|w| <= 1/sqrt(fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    shapes = [(128, 256), (256,)] + [(256, 256), (256,)] * 3 + [(256, 3), (3,)]
    parts = [rng.uniform(-1, 1, s) / math.sqrt(s[0]) if len(s) == 2 else np.zeros(s) for s in shapes]
    p = np.concatenate([x.ravel() for x in parts]).astype(np.float32)
    assert p.size == lcs.LCS_MLP_PARAMS
    return p


def new_model(cfg: SurrogateConfig, device="cuda") -> lcs.Mlp:
    return lcs.Mlp(init_params(cfg.seed + 1), make_frequencies(cfg),
                   in_shift=[0.0, 0.0, 0.0, cfg.t0],
                   in_scale=[1.0 / cfg.period] * 3 + [1.0 / (cfg.n_windows * cfg.tau)],
                   out_scale=cfg.tau * cfg.speed_scale, device=device)


def training_data(frames: lcs.DeviceFrames, cfg: SurrogateConfig, n: int, seed: int = 0):
    """n pairs (x0, t0) -> RK4 displacement over tau: x0 uniform on the torus,
    t0 uniform on cfg.t0_choices."""
    torch = lcs._torch()
    dev = frames.u[0].device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    x0 = torch.rand((3, n), generator=gen, device=dev, dtype=torch.float32) * float(cfg.period)
    choices = torch.tensor(list(cfg.t0_choices), dtype=torch.float64, device=dev)
    t0 = choices[torch.randint(len(cfg.t0_choices), (n,), generator=gen, device=dev)]
    xf, _, flags = lcs.lcs_advect_points(frames, x0, t0, cfg.tau, cfg.dt, want_cell=False)
    dx = lcs.lcs_sub(xf, x0)
    xt = torch.empty((4, n), dtype=torch.float32, device=dev)
    xt[:3] = x0
    xt[3] = t0.to(torch.float32)
    return xt, dx, flags


@dataclass
class TrainLog:
    steps: int = 0
    seconds: float = 0.0
    losses: list = field(default_factory=list)
    val_loss: Optional[float] = None


def train(mlp: lcs.Mlp, xt, dx, epochs: int, batch: int = 65536, lr: float = 2e-3,
          lr_final: float = 1e-4, val=None, log_every: int = 50) -> TrainLog:
    """Adam on the MSE of the displacement, cosine learning-rate decay: one
    lcs_mlp_train call runs every step (batches in order, epoch after epoch)."""
    torch = lcs._torch()
    n = int(xt.shape[1])
    nb = n // batch
    total = epochs * nb
    m = torch.zeros_like(mlp.params)
    v = torch.zeros_like(mlp.params)
    losses = torch.empty(total, dtype=torch.float64, device=xt.device)
    ws = torch.empty(lcs.lcs_mlp_train_workspace_bytes(batch), dtype=torch.uint8, device=xt.device)
    log = TrainLog()
    torch.cuda.synchronize()
    t = time.perf_counter()
    lcs.lcs_mlp_train(mlp, xt, dx, batch, 1, total, total, m, v, lr=lr, lr_final=lr_final,
                      losses=losses, workspace=ws)
    torch.cuda.synchronize()
    log.seconds = time.perf_counter() - t
    log.steps = total
    lh = losses.cpu().numpy()
    log.losses = [(k, float(lh[k - 1])) for k in range(1, total + 1) if k % log_every == 0 or k == total]
    if val is not None:
        log.val_loss = evaluate(mlp, *val)
    return log


def evaluate(mlp: lcs.Mlp, xt, dx, batch: int = 1 << 20) -> float:
    """Mean squared displacement error over a held-out set."""
    torch = lcs._torch()
    n = int(xt.shape[1])
    tot = 0.0
    for s in range(0, n, batch):
        e = min(n, s + batch)
        out, _ = lcs.lcs_mlp_forward(mlp, xt[:, s:e].contiguous())
        _, l = lcs.lcs_mse_grad(out, dx[:, s:e].contiguous(), want_grad=False)
        tot += float(l.item()) * (e - s)
    return tot / n


def surrogate_flowmap(mlp: lcs.Mlp, frames: lcs.DeviceFrames, seeds, cfg: SurrogateConfig,
                      tol: float, full_fallback_fraction: float = 0.25, workspace=None,
                      stream=None):
    """Composed surrogate flow map with RK4 check samples and RK4 fallback on
    failing tiles (lcs_surrogate_flowmap; the fallback policy is the
    library's: more than ``full_fallback_fraction`` of the tiles failing
    re-advects the whole grid).  Returns (xf, flags, n_fail, tile_err)."""
    xf, flags, nf, _, err = lcs.lcs_surrogate_flowmap(
        mlp, frames, seeds, cfg.t0, cfg.tau, cfg.n_windows, tol, cfg.dt,
        whole_grid_fraction=full_fallback_fraction, workspace=workspace, stream=stream)
    return xf, flags, nf, err


def save(mlp: lcs.Mlp, cfg: SurrogateConfig, path: str):
    d = mlp.desc
    np.savez(path, params=mlp.params.cpu().numpy(), freq=mlp.freq.cpu().numpy(),
             in_shift=np.array(list(d.in_shift), np.float32),
             in_scale=np.array(list(d.in_scale), np.float32),
             out_scale=np.float32(d.out_scale), tau=cfg.tau, n_windows=cfg.n_windows, t0=cfg.t0)


def load(path: str, device="cuda") -> lcs.Mlp:
    z = np.load(path, allow_pickle=False)
    return lcs.Mlp(z["params"], z["freq"], z["in_shift"], z["in_scale"], float(z["out_scale"]),
                   device=device)
