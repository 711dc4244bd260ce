"""Autotuner for the advection launch: picks the seed-ordering strategy.

Candidates (all produce bit-identical results, only speed differs):
  * "tiles"      -- lcs_advect: one launch, seeds in Morton-ordered workgroup
                    tiles for the whole integration;
  * "sorted:S"   -- lcs_advect_sorted with segments of S RK4 steps: tracers are
                    re-bundled by position between segments.
Each candidate is timed on the caller's workload (events on the stream the
work runs on) and the fastest is cached in a JSON file keyed by the workload
signature and the GPU architecture.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional

from . import lcs

DEFAULT_CANDIDATES = ("tiles", "sorted:200", "sorted:100", "sorted:50", "sorted:25")


def signature(frames: lcs.DeviceFrames, seeds, t0: float, T: float, dt: float) -> str:
    d = frames.desc
    dims = "x".join(str(int(d.n[a])) for a in range(d.dim))
    sd = "x".join(str(int(seeds.n[a])) for a in range(seeds.dim))
    return (f"{d.dim}d:grid{dims}:per{int(d.periodic_mask)}:frames{int(d.n_frames)}:seeds{sd}:"
            f"steps{int(round(T / dt))}")


def _arch() -> str:
    torch = lcs._torch()
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def run(choice: str, frames, seeds, t0, T, dt, xf=None, cell=None, flags=None, workspace=None,
        want_cell=True, stream=None):
    """Run the advection with one candidate strategy."""
    if choice == "tiles":
        return lcs.lcs_advect(frames, seeds, t0, T, dt, xf, cell, flags, want_cell=want_cell,
                              stream=stream)
    seg = int(choice.split(":")[1])
    return lcs.lcs_advect_sorted(frames, seeds, t0, T, dt, seg, xf, cell, flags, workspace,
                                 want_cell=want_cell, stream=stream)


def tune(frames, seeds, t0, T, dt, candidates: Iterable[str] = DEFAULT_CANDIDATES,
         cache_path: Optional[str] = None, stream=None) -> Dict:
    """Time every candidate once (after one untimed run of the first) and
    return {"choice": best, "ms": {candidate: ms}}; cached when a path is given."""
    torch = lcs._torch()
    key = f"{_arch()}:{signature(frames, seeds, t0, T, dt)}"
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]
    stream = stream or torch.cuda.current_stream()
    dev = frames.u[0].device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    xf = torch.empty((seeds.dim, ns), dtype=torch.float32, device=dev)
    flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    ws = None
    if any(c != "tiles" for c in candidates):
        ws = torch.empty(lcs.lcs_advect_sorted_workspace_bytes(frames, seeds), dtype=torch.uint8,
                         device=dev)
    cands = list(candidates)
    run(cands[0], frames, seeds, t0, T, dt, xf, None, flags, ws, want_cell=False, stream=stream)
    times = {}
    for c in cands:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        run(c, frames, seeds, t0, T, dt, xf, None, flags, ws, want_cell=False, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        times[c] = e0.elapsed_time(e1)
    best = min(times, key=times.get)
    rec = {"choice": best, "ms": times}
    if cache_path:
        cache[key] = rec
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return rec
