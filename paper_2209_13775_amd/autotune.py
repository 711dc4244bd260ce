"""Seed-ordering autotuner (Python face of the library's lcs_advect_tuned).

Candidates (all produce bit-identical results, only speed differs):
  * "tiles"      -- lcs_advect: one launch, seeds in Morton-ordered workgroup
                    tiles for the whole integration;
  * "sorted:S"   -- lcs_advect_sorted with segments of S RK4 steps: tracers are
                    re-bundled by position between segments.
The timing, the choice and the cache file are the library's (a plan created
with an autotune cache path); this module only names the candidates.
"""
from __future__ import annotations

from typing import Dict, Iterable, Optional

from . import lcs

DEFAULT_CANDIDATES = ("tiles", "sorted:200", "sorted:100", "sorted:50", "sorted:25")


def _seg(choice: str) -> int:
    return 0 if choice == "tiles" else int(choice.split(":")[1])


def _name(seg: int) -> str:
    return "tiles" if seg == 0 else f"sorted:{seg}"


def run(choice: str, frames, seeds, t0, T, dt, xf=None, cell=None, flags=None, workspace=None,
        want_cell=True, stream=None):
    """Run the advection with one candidate strategy."""
    if choice == "tiles":
        return lcs.lcs_advect(frames, seeds, t0, T, dt, xf, cell, flags, want_cell=want_cell,
                              stream=stream)
    return lcs.lcs_advect_sorted(frames, seeds, t0, T, dt, _seg(choice), xf, cell, flags,
                                 workspace, want_cell=want_cell, stream=stream)


def tune(frames, seeds, t0, T, dt, candidates: Iterable[str] = DEFAULT_CANDIDATES,
         cache_path: Optional[str] = None, stream=None) -> Dict:
    """Let the library time the candidates on this workload (once per workload
    key; cached in ``cache_path`` when given) and return
    {"choice": best, "ms": {candidate: ms} or None when the cache answered}."""
    torch = lcs._torch()
    cands = list(candidates)
    dev = frames.u[0].device
    ns = int(seeds.n[0] * seeds.n[1] * seeds.n[2])
    ws = None
    if any(c != "tiles" for c in cands):
        ws = torch.empty(lcs.lcs_advect_sorted_workspace_bytes(frames, seeds), dtype=torch.uint8,
                         device=dev)
    xf = torch.empty((seeds.dim, ns), dtype=torch.float32, device=dev)
    plan = lcs.Plan(autotune_cache=cache_path)
    try:
        _, _, _, seg, ms = lcs.lcs_advect_tuned(plan, frames, seeds, t0, T, dt, xf=xf,
                                                workspace=ws, candidates=[_seg(c) for c in cands],
                                                want_cell=False, want_flags=False, stream=stream)
        torch.cuda.synchronize()
    finally:
        plan.close()
    return {"choice": _name(seg),
            "ms": None if ms is None else {_name(k): v for k, v in ms.items()}}
