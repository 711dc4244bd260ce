"""lcs_advect_sorted_noalloc (workspace in the library's fixed device array,
nothing allocated by the call) against lcs_advect_sorted, through the C ABI:
two calls in a row, the second on a smaller grid, each bit-identical to the
caller-workspace entry point; a grid needing more scratch than the array is
refused on the host."""
import ctypes as C
import math
import sys

import numpy as np
import pytest

from paper_2209_13775_amd import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_noalloc_matches_sorted_twice_then_smaller():
    import torch
    assert torch.cuda.is_available()
    from paper_2209_13775_amd import lcs
    L = 2 * math.pi
    fs = inputs.abc_frames(n=32, n_frames=17, dt_frame=0.5)
    frames = lcs.DeviceFrames(fs)
    for n in [(45, 38, 29), (21, 17, 9)]:
        g = inputs.periodic_seeds(3, n, (L, L, L))
        ns = g.count
        _say(f"case: no-alloc re-bundled advection, seeds {n}")
        ref = lcs.lcs_advect_sorted(frames, g, 8.0, -6.0, -0.02, segment_steps=37)
        xf = torch.full((3, ns), float("nan"), dtype=torch.float32, device="cuda")
        cell = torch.full((ns,), -7, dtype=torch.int64, device="cuda")
        flags = torch.full((ns,), 99, dtype=torch.uint8, device="cuda")
        lcs.lcs_advect_sorted_noalloc(frames, g, 8.0, -6.0, -0.02, 37, xf, cell, flags)
        lcs.lcs_sync_status()
        assert torch.equal(xf, ref[0]) and torch.equal(cell, ref[1]) and torch.equal(flags, ref[2])
    # a 2D grid with flagged tracers (a NaN frame node) after the 3D calls (the
    # array keeps their contents)
    fs2 = inputs.double_gyre_frames(nx=101, ny=51, n_frames=21)
    fs2.u[0][5, 20, 40] = np.nan
    frames2 = lcs.DeviceFrames(fs2)
    g2 = inputs.linspace_seeds(2, (150, 71), (0.0, 0.0), (2.0, 1.0))
    _say("case: no-alloc re-bundled advection, 2D with flagged tracers")
    ref = lcs.lcs_advect_sorted(frames2, g2, 0.0, 10.0, 0.05, segment_steps=50)
    xf = torch.empty((2, g2.count), dtype=torch.float32, device="cuda")
    flags = torch.empty(g2.count, dtype=torch.uint8, device="cuda")
    lcs.lcs_advect_sorted_noalloc(frames2, g2, 0.0, 10.0, 0.05, 50, xf, None, flags)
    lcs.lcs_sync_status()
    assert int((flags != 0).sum()) > 0
    assert torch.equal(xf, ref[0]) and torch.equal(flags, ref[2])


def test_noalloc_refuses_grids_beyond_its_scratch():
    import torch
    from paper_2209_13775_amd import lcs
    L = 2 * math.pi
    fs = inputs.abc_frames(n=16, n_frames=5, dt_frame=0.5)
    frames = lcs.DeviceFrames(fs)
    g = inputs.periodic_seeds(3, (128, 128, 128), (L, L, L))      # ~2M seeds, > 64 MiB
    assert lcs.lcs_advect_sorted_workspace_bytes(frames, g) > lcs.LCS_NOALLOC_SCRATCH_BYTES
    sd = lcs.seed_grid_desc(g)
    st = lcs.lib().lcs_advect_sorted_noalloc(frames.ref, C.byref(sd), 0.0, 1.0, 0.1, 0,
                                             C.c_void_p(0x10), None, None, None)
    assert st == lcs.LCS_E_SHAPE and "scratch" in lcs.lcs_last_error()
