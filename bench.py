"""Benchmark of the LCS hot path on one MI355X.

One step = the whole hot path over one batch of synthetic input:
lcs_advect (seed grid -> RK4 flow map) -> lcs_cg_tensor (grad F, C) ->
lcs_ftle (lambda_max, FTLE), on the time-dependent ABC flow sampled on a
128^3 periodic grid (33 FP32 frames, t in [0, 16]) with 256^3 seeds,
t0 = 0, T = 8, dt = 0.02 (400 RK4 steps).

Prints one JSON line.  ``value`` is tracer-RK4-steps per second of the whole
step; the roofline object covers the advection kernel (the dominant one),
timed with events on the stream it is launched on; the CPU baseline is the
FP64 oracle on a bounded sample of the same seeds, on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
BYTES_PER_STEP_3D = 768      # 4 evals x 8 corners x 2 frames x 3 comps x 4 B
WORKLOAD = dict(name="abc_128cubed_seeds256cubed", grid=128, frames=33, dt_frame=0.5,
                seeds=(256, 256, 256), t0=0.0, T=8.0, dt=0.02)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target wall time of the oracle sample")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched-window, random-Fourier and surrogate workloads")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate workload")
    ap.add_argument("--layout", default="tpair", choices=("soa", "xyz", "xyzw", "tpair"),
                    help="frame layout the kernels read; with an interleaved layout the main "
                         "step converts the structure-of-arrays frames inside its timed region")
    ap.add_argument("--extras", default="batched,random_fourier,surrogate,mesh,ab,aux,time_resolved",
                    help="comma-separated extra workloads to run after the main step")
    ap.add_argument("--strategy", default=None,
                    help="advection strategy of the main workload ('tiles' or 'sorted:S'); "
                         "default: autotuned")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB, so that "
                         "profiler byte counters can be scaled by a kernel of known traffic")
    return ap.parse_args()


PROFILES = os.path.join(ROOT, "profiles")


def source_hash(files):
    """SHA-1 (16 hex digits) of kernel sources with comments and blank lines
    removed: the code the counters were taken on, not its commentary."""
    import hashlib
    import re
    h = hashlib.sha1()
    for f in files:
        text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, f)).read(), flags=re.S)
        for line in text.splitlines():
            line = re.sub(r"//.*$", "", line).strip()
            if line:
                h.update(line.encode() + b"\n")
    return h.hexdigest()[:16]


def profiled_traffic_kernel(kernel):
    """HBM bytes per launch of a kernel from its committed rocprofv3 counter
    summary, or None if there is none or its source changed since."""
    try:
        names = sorted(os.listdir(PROFILES))
    except OSError:
        return None
    for name in names:
        if not name.endswith(".md"):
            continue
        for line in open(os.path.join(PROFILES, name)).read().splitlines():
            if not (line.startswith("{") and "traffic_bytes_per_launch" in line):
                continue
            rec = json.loads(line)
            if rec.get("kernel") != kernel:
                continue
            if source_hash(rec["source_files"]) == rec["source_sha1"]:
                return rec["traffic_bytes_per_launch"]
    return None


# frame layout of the 3D workloads (set from --layout in main)
LAYOUT_3D = "tpair"


def stage_frames(lcs, fs, layout, tensors=None):
    """Device frames of fs in the given layout (interleaved copies are made by
    lcs_frames_interleave from the structure-of-arrays frames)."""
    soa = lcs.DeviceFrames(fs, tensors=tensors)
    if layout == "soa":
        return soa
    fr = lcs.lcs_frames_interleave(soa, layout)
    del soa
    return fr


def profiled_traffic(strategy, layout="soa"):
    """HBM bytes of one advection call (all its kernels) from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, each scaled by a plain
    copy of known size), or None if it was taken for another strategy or the
    kernel source changed since."""
    try:
        names = sorted(os.listdir(PROFILES))
    except OSError:
        return None
    for name in names:
        if not name.endswith(".md"):
            continue
        for line in open(os.path.join(PROFILES, name)).read().splitlines():
            if not (line.startswith("{") and "traffic_bytes_per_launch" in line):
                continue
            rec = json.loads(line)
            if rec.get("strategy", "tiles") != strategy or rec.get("layout", "soa") != layout:
                continue
            if source_hash(rec["source_files"]) == rec["source_sha1"]:
                return rec["traffic_bytes_per_launch"]
    return None


def profiled_counter(kernel, field):
    """A figure (l2_hit_rate, ta_busy, td_busy, ...) of a kernel from the
    committed rocprofv3 counter summary, or None if there is none or its
    source changed since."""
    try:
        names = sorted(os.listdir(PROFILES))
    except OSError:
        return None
    for name in names:
        if not name.endswith(".md"):
            continue
        for line in open(os.path.join(PROFILES, name)).read().splitlines():
            if not (line.startswith("{") and f'"{field}"' in line):
                continue
            rec = json.loads(line)
            if rec.get("kernel") == kernel and \
                    source_hash(rec["source_files"]) == rec["source_sha1"]:
                return rec[field]
    return None


def measure_copy_gbs(torch, dev, mib=1024, reps=5):
    """Device-to-device copy rate (bytes read + written per second) of a plain
    torch copy of mib MiB: the HBM rate this device reaches in practice."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def cpu_baseline(fs, g, t0, T, dt, target_s):
    """FP64 oracle on a bounded, deterministic sample of the seeds."""
    import oracle
    vel = oracle.Velocity(fs)
    threads = oracle.default_threads()
    nsteps = int(round(T / dt))
    rng = np.random.default_rng(0)
    m = 4096
    idx = np.sort(rng.choice(g.count, size=m, replace=False))
    t = time.perf_counter()
    oracle.advect_seeds(vel, g, t0, T, dt, idx=idx, threads=threads)
    el = time.perf_counter() - t
    m2 = int(min(g.count, max(m, m * target_s / max(el, 1e-3))))
    if m2 > m * 1.5:
        idx = np.sort(rng.choice(g.count, size=m2, replace=False))
        t = time.perf_counter()
        oracle.advect_seeds(vel, g, t0, T, dt, idx=idx, threads=threads)
        el = time.perf_counter() - t
        m = m2
    # one thread as well, the serial baseline the paper compares with
    m1 = max(64, int(m * 2.0 / max(el * threads, 1e-3)))
    idx1 = np.sort(rng.choice(g.count, size=m1, replace=False))
    t = time.perf_counter()
    oracle.advect_seeds(vel, g, t0, T, dt, idx=idx1, threads=1)
    el1 = time.perf_counter() - t
    return {"value": m * nsteps / el, "unit": "tracer-RK4-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{m} seeds drawn from the 256^3 grid (seed 0), full T=8 ({nsteps} RK4 steps), "
                      f"FP64, OpenMP, {el:.1f} s",
            "single_thread_value": m1 * nsteps / el1,
            "single_thread_sample": f"{m1} seeds, full T, one thread, {el1:.1f} s",
            "cpu_model": cpu_model()}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_batched(torch, lcs, inputs, reps=3, layout="xyz"):
    """Double gyre on 1025x513 nodes x 101 FP32 frames (t = 0.25 f); 64 windows
    (t0 ~ U[0,10], T from {5, 7.5, 10, 12.5, 15}, default_rng(0)) of a
    1024x512 seed grid, dt = 0.05, all in one graph-replayed persistent launch."""
    fs = inputs.double_gyre_frames(nx=1025, ny=513, n_frames=101, dt_frame=0.25,
                                   dtype=np.float32)
    g = inputs.linspace_seeds(2, (1024, 512), (0.0, 0.0), (2.0, 1.0))
    windows = inputs.t0_windows(64, seed=0)
    dt = 0.05
    frames = stage_frames(lcs, fs, layout)
    plan = lcs.Plan()
    nw, ns = len(windows), g.count
    xf = torch.empty((nw, 2, ns), dtype=torch.float32, device="cuda")
    cell = torch.empty((nw, ns), dtype=torch.int64, device="cuda")
    flags = torch.empty((nw, ns), dtype=torch.uint8, device="cuda")
    lcs.lcs_advect_batched(plan, frames, g, windows, dt, xf, cell, flags)   # capture + warm-up
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lcs.lcs_advect_batched(plan, frames, g, windows, dt, xf, cell, flags, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    lcs.lcs_sync_status()
    steps = int(sum(round(T / dt) for _, T in windows)) * ns
    ms = float(np.median(times))
    out = {"workload": "double_gyre_batched_1025x513_64windows", "frame_layout": layout,
           "windows": nw,
           "seeds_per_window": ns, "tracer_steps": steps, "ms_per_launch": ms,
           "tracer_steps_per_s": steps / (ms * 1e-3),
           "roofline": {"kernel": "advect_batched_kernel<2>", "bound": "hbm",
                        "achieved": 256 * steps / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": 256 * steps / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "bytes_per_unit": 256, "unit_of_work": "2D tracer-RK4-step"},
           "graph": plan.stats()}
    plan.close()
    return out


def bench_random_fourier(torch, lcs, inputs, reps=1, keep=None):
    """Divergence-free random-Fourier field, 256^3 x 65 FP32 frames, 512x512x256
    seeds, forward and backward FTLE from t0 = 4 with |T| = 4, dt = 0.01."""
    fs = inputs.random_fourier_frames(n=256, n_frames=65, dt_frame=0.125, device="cuda")
    L = 2 * math.pi
    g = inputs.SeedGrid(3, (512, 512, 256), (0.0, 0.0, 0.0), (L / 512, L / 512, L / 256),
                        (True, True, True))
    frames = stage_frames(lcs, fs, LAYOUT_3D, tensors=fs.u)
    ns = g.count
    from paper_2209_13775_amd import autotune
    tuned = autotune.tune(frames, g, 4.0, 4.0, 0.01, candidates=("sorted:100", "sorted:50",
                                                                    "sorted:25"))
    choice = tuned["choice"]
    ws = torch.empty(lcs.lcs_advect_sorted_workspace_bytes(frames, g), dtype=torch.uint8,
                     device="cuda")
    xf = torch.empty((3, ns), dtype=torch.float32, device="cuda")
    flags = torch.empty(ns, dtype=torch.uint8, device="cuda")
    lam = torch.empty(ns, dtype=torch.float64, device="cuda")
    sig = torch.empty(ns, dtype=torch.float64, device="cuda")
    sfl = torch.empty(ns, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    res = {}
    for T, dt in [(4.0, 0.01), (-4.0, -0.01)]:
        ta, tc = [], []
        for _ in range(reps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            autotune.run(choice, frames, g, 4.0, T, dt, xf, None, flags, ws, want_cell=False,
                         stream=stream)
            e[1].record(stream)
            lcs.lcs_cg_ftle(g, xf, T, flags=flags, lambda_max=lam, ftle=sig, stencil_flags=sfl,
                            stream=stream)
            e[2].record(stream)
            torch.cuda.synchronize()
            ta.append(e[0].elapsed_time(e[1]))
            tc.append(e[1].elapsed_time(e[2]))
        res["forward" if T > 0 else "backward"] = (float(np.median(ta)), float(np.median(tc)),
                                                   float(sig.mean().item()))
        if T > 0 and keep is not None:
            keep.update(fs=fs, frames=frames, seeds=g, ref_ftle=sig.clone(),
                        rk4_ms=float(np.median(ta)) + float(np.median(tc)))
    lcs.lcs_sync_status()
    nsteps = 400
    steps = 2 * ns * nsteps
    adv = res["forward"][0] + res["backward"][0]
    cgf = res["forward"][1] + res["backward"][1]
    del ws
    return {"workload": "random_fourier_256cubed_seeds512x512x256", "frame_layout": LAYOUT_3D,
            "seeds": ns,
            "advect_strategy": choice, "autotune_ms": tuned["ms"],
            "tracer_steps": steps, "advect_ms_forward": res["forward"][0],
            "advect_ms_backward": res["backward"][0], "cg_ftle_ms": cgf,
            "tracer_steps_per_s": steps / ((adv + cgf) * 1e-3),
            "ftle_points_per_s": 2 * ns / (cgf * 1e-3),
            "mean_ftle_forward": res["forward"][2], "mean_ftle_backward": res["backward"][2],
            "roofline": {"kernel": "advection call (%s)" % choice, "bound": "hbm",
                         "achieved": 768 * steps / (adv * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": 768 * steps / (adv * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "bytes_per_unit": 768, "unit_of_work": "3D tracer-RK4-step"}}


MESH_BYTES_PER_STEP_3D = 640   # 4 x (cell map 48 B + node ids 16 B + 2 frames x 4 nodes x 12 B)
MESH_BYTES_PER_STEP_2D = 256   # 4 x (cell map 24 B + node ids 16 B + 2 frames x 3 nodes x 8 B)


def bench_mesh(torch, lcs, inputs, reps=3, cpu_sample=0):
    """Velocity on unstructured meshes: the 3D workload (time-dependent cellular
    box flow on 64^3 x 6 jittered tetrahedra, 192^3 seeds, T = 8, dt = 0.02) and
    the 2D one (double gyre on 200 x 100 x 2 jittered triangles, 256 x 128
    seeds, T = 10, dt = 0.05)."""
    out = {}
    cases = [("box_cells_tetmesh_64cubed_x6_seeds192cubed", 3),
             ("double_gyre_trimesh_200x100x2_seeds256x128", 2)]
    for name, dim in cases:
        w = inputs.WORKLOADS[name]
        if dim == 3:
            mf = inputs.box_cells_mesh_frames(cells=w["cells"], n_frames=w["frames"],
                                              dt_frame=w["dt_frame"])
            g = inputs.linspace_seeds(3, w["seeds"], (0.0,) * 3, (math.pi,) * 3)
        else:
            mf = inputs.double_gyre_mesh_frames(w["cells"], n_frames=w["frames"],
                                                dt_frame=w["dt_frame"])
            g = inputs.linspace_seeds(2, w["seeds"], (0.0, 0.0), (2.0, 1.0))
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        t = time.perf_counter()
        gm = lcs.Mesh(mf.mesh, stream=stream)
        torch.cuda.synchronize()
        create_ms = (time.perf_counter() - t) * 1e3
        fr = lcs.MeshFrames(mf)
        ns = g.count
        xf = torch.empty((dim, ns), dtype=torch.float32, device="cuda")
        cell = torch.empty(ns, dtype=torch.int64, device="cuda")
        flags = torch.empty(ns, dtype=torch.uint8, device="cuda")
        sig = torch.empty(ns, dtype=torch.float64, device="cuda")
        t0, T, dt = w["t0"], w["T"], w["dt"]
        lcs.lcs_mesh_advect(gm, fr, g, t0, T, dt, xf, cell, flags, stream=stream)
        ta, tc = [], []
        for _ in range(reps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            lcs.lcs_mesh_advect(gm, fr, g, t0, T, dt, xf, cell, flags, stream=stream)
            e[1].record(stream)
            lcs.lcs_cg_ftle(g, xf, T, flags=flags, ftle=sig, stream=stream)
            e[2].record(stream)
            torch.cuda.synchronize()
            ta.append(e[0].elapsed_time(e[1]))
            tc.append(e[1].elapsed_time(e[2]))
        lcs.lcs_sync_status()
        adv, cgf = float(np.median(ta)), float(np.median(tc))
        steps = ns * int(round(T / dt))
        bps = MESH_BYTES_PER_STEP_3D if dim == 3 else MESH_BYTES_PER_STEP_2D
        fl = flags.cpu().numpy()
        c = g.coords_of(np.arange(ns))
        on_wall = np.zeros(ns, dtype=bool)
        for a in range(dim):
            on_wall |= (c[a] == 0) | (c[a] == g.n[a] - 1)
        rec = {"workload": name, "cells": gm.n_cells, "nodes": gm.n_nodes, "seeds": ns,
               "flagged_wall_seeds": int(((fl != 0) & on_wall).sum()),
               "flagged_interior_seeds": int(((fl != 0) & ~on_wall).sum()),
               "mesh_create_ms": create_ms, "advect_ms": adv, "cg_ftle_ms": cgf,
               "tracer_steps": steps, "tracer_steps_per_s": steps / ((adv + cgf) * 1e-3),
               "tracer_steps_per_s_advect_kernel": steps / (adv * 1e-3),
               "ftle_points_per_s": ns / (cgf * 1e-3), "mean_ftle": float(sig.mean().item()),
               "flagged_tracers": int((fl != 0).sum()), "lost_tracers": int(((fl & 16) != 0).sum()),
               "roofline": {"kernel": "mesh_advect_grid_kernel<%d>" % dim, "bound": "hbm",
                            "achieved": bps * steps / (adv * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s",
                            "frac": bps * steps / (adv * 1e-3) / 1e9 / HBM_PEAK_GBS,
                            "traffic": profiled_traffic_kernel("mesh_advect_grid_kernel<%d>" % dim),
                            "bytes_per_unit": bps, "unit_of_work": "%dD mesh tracer-RK4-step" % dim}}
        if cpu_sample and dim == 3:
            import oracle
            mv = oracle.MeshVelocity(mf)
            idx = np.random.default_rng(0).choice(ns, size=cpu_sample, replace=False)
            thr = oracle.default_threads()
            t = time.perf_counter()
            mv.advect_seeds(g, t0, T, dt, idx=idx, threads=thr)
            sec = time.perf_counter() - t
            rec["cpu_baseline"] = {"value": cpu_sample * int(round(T / dt)) / sec,
                                   "unit": "tracer-RK4-steps/s", "cores": thr, "kind": "oracle",
                                   "sample": "%d seeds drawn from the grid (seed 0), full T, FP64, "
                                             "%.1f s" % (cpu_sample, sec)}
        out[name] = rec
        gm.close()
        del fr, xf, cell, flags, sig
        torch.cuda.empty_cache()
    return out


def bench_ab(torch, lcs, inputs, reps=2):
    """Adams-Bashforth (AB4, RK4 start-up) on the ABC 128^3 / 256^3-seed / T = 8
    workload: time per call and FTLE error against a fine-step RK4 reference
    (dt = 0.005), beside RK4 at the benchmark step dt = 0.02."""
    fs = inputs.abc_frames(n=128, n_frames=33, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (256, 256, 256), (L, L, L))
    frames = stage_frames(lcs, fs, LAYOUT_3D)
    ns = g.count
    T = 8.0
    stream = torch.cuda.current_stream()
    xf = torch.empty((3, ns), dtype=torch.float32, device="cuda")
    flags = torch.empty(ns, dtype=torch.uint8, device="cuda")
    sig = torch.empty(ns, dtype=torch.float64, device="cuda")
    ws = torch.empty(lcs.lcs_advect_sorted_workspace_bytes(frames, g), dtype=torch.uint8,
                     device="cuda")
    lcs.lcs_advect_sorted(frames, g, 0.0, T, 0.005, 200, xf, None, flags, ws, want_cell=False,
                          stream=stream)
    lcs.lcs_cg_ftle(g, xf, T, flags=flags, ftle=sig, stream=stream)
    ref = sig.clone()

    def timed(fn):
        fn()
        ms = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        lcs.lcs_cg_ftle(g, xf, T, flags=flags, ftle=sig, stream=stream)
        err = (sig - ref).abs()
        return float(np.median(ms)), float(err.mean().item()), float(err.max().item())

    runs = []
    ms, em, ex = timed(lambda: lcs.lcs_advect_sorted(frames, g, 0.0, T, 0.02, 100, xf, None, flags,
                                                     ws, want_cell=False, stream=stream))
    runs.append({"method": "rk4 (re-bundled, segments of 100)", "dt": 0.02, "ms": ms,
                 "ftle_err_mean": em, "ftle_err_max": ex})
    ms, em, ex = timed(lambda: lcs.lcs_advect_ab(frames, g, 0.0, T, 0.02, order=4, xf=xf,
                                                 want_cell=False, flags=flags, stream=stream))
    runs.append({"method": "ab4 (single launch)", "dt": 0.02, "ms": ms, "ftle_err_mean": em,
                 "ftle_err_max": ex})
    del ws
    ws = torch.empty(lcs.lcs_advect_ab_sorted_workspace_bytes(frames, g), dtype=torch.uint8,
                     device="cuda")
    ab_ms = None
    for dt in (0.02, 0.01, 0.005):
        seg = int(round(2.0 / dt))
        ms, em, ex = timed(lambda: lcs.lcs_advect_ab_sorted(
            frames, g, 0.0, T, dt, order=4, segment_steps=seg, xf=xf, flags=flags, workspace=ws,
            want_cell=False, stream=stream))
        if dt == 0.02:
            ab_ms = ms
        runs.append({"method": "ab4 (re-bundled every 2.0 time units)", "dt": dt, "ms": ms,
                     "ftle_err_mean": em, "ftle_err_max": ex})
    lcs.lcs_sync_status()
    steps = ns * 400
    del ws, frames
    return {"workload": "abc_128cubed_seeds256cubed_ab4", "frame_layout": LAYOUT_3D,
            "reference": "rk4 dt=0.005",
            "runs": runs, "tracer_steps_per_s_ab4_dt0.02": steps / (ab_ms * 1e-3),
            "velocity_evaluations_per_step": {"rk4": 4, "ab4": 1},
            "roofline": {"kernel": "ab4 re-bundled call (rebundle_segment_kernel<3, 4> + sorts)",
                         "bound": "hbm",
                         "achieved": 192 * steps / (ab_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": 192 * steps / (ab_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "bytes_per_unit": 192, "unit_of_work": "3D tracer-AB4-step"}}


def bench_aux(torch, lcs, inputs, reps=2):
    """Auxiliary-point gradient against seed-grid differences on the ABC field
    (128^3 nodes, T = 8, dt = 0.02), FTLE at 128^3 seeds: error of (a) grid
    differences on the 128^3 seeds, (b) grid differences on 256^3 seeds read at
    the same points, (c) auxiliary points with delta = h/10 -- each against
    auxiliary points with delta = h/100 -- and the time of each."""
    fs = inputs.abc_frames(n=128, n_frames=33, dt_frame=0.5)
    L = 2 * math.pi
    g = inputs.periodic_seeds(3, (128, 128, 128), (L, L, L))
    g2 = inputs.periodic_seeds(3, (256, 256, 256), (L, L, L))
    frames = stage_frames(lcs, fs, LAYOUT_3D)
    T, dt = 8.0, 0.02
    h = L / 128
    stream = torch.cuda.current_stream()

    def timed(fn):
        out = fn()
        ms = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            out = fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return out, float(np.median(ms))

    # every variant re-bundled, segments of 100 steps
    ws = torch.empty(max(lcs.lcs_advect_aux_sorted_workspace_bytes(frames, g),
                         lcs.lcs_advect_sorted_workspace_bytes(frames, g2)),
                     dtype=torch.uint8, device="cuda")

    def aux(delta):
        hi, lo, fl = lcs.lcs_advect_aux_sorted(frames, g, [delta] * 3, 0.0, T, dt, 100,
                                               workspace=ws, stream=stream)
        Cm, sfl = lcs.lcs_cg_aux(g, [delta] * 3, hi, lo, fl, stream=stream)
        _, sig = lcs.lcs_ftle(3, Cm, T, want_lambda=False, stream=stream)
        return sig

    def grid(gg):
        xf, _, fl = lcs.lcs_advect_sorted(frames, gg, 0.0, T, dt, 100, workspace=ws, want_cell=False,
                                          stream=stream)
        _, sig, _ = lcs.lcs_cg_ftle(gg, xf, T, flags=fl, stream=stream)
        return sig

    ref, ms_ref = timed(lambda: aux(h / 100))
    s_aux, ms_aux = timed(lambda: aux(h / 10))
    s_g1, ms_g1 = timed(lambda: grid(g))
    s_g2, ms_g2 = timed(lambda: grid(g2))
    s_g2 = s_g2.reshape(256, 256, 256)[::2, ::2, ::2].reshape(-1)
    lcs.lcs_sync_status()

    def err(x):
        e = (x - ref).abs()
        return {"ftle_err_mean": float(e.mean().item()), "ftle_err_p99": float(torch.quantile(
            e[::17].float(), 0.99).item()), "ftle_err_max": float(e.max().item())}

    ns = g.count
    return {"workload": "abc_128cubed_ftle_at_128cubed_seeds_aux_vs_grid", "frame_layout": LAYOUT_3D,
            "advect_strategy": "re-bundled, segments of 100 (lcs_advect_aux_sorted, lcs_advect_sorted)",
            "reference":
            "auxiliary points, delta = h/100", "seed_spacing_h": h,
            "grid_128cubed": dict(ms=ms_g1, tracers=ns, **err(s_g1)),
            "grid_256cubed_subsampled": dict(ms=ms_g2, tracers=8 * ns, **err(s_g2)),
            "aux_delta_h_over_10": dict(ms=ms_aux, tracers=6 * ns, **err(s_aux)),
            "aux_reference_ms": ms_ref,
            "aux_tracer_steps_per_s": 6 * ns * 400 / (ms_aux * 1e-3)}


def bench_time_resolved(torch, lcs, inputs, reps=2):
    """Time-resolved FTLE on the ABC 128^3 / 256^3-seed workload (8 snapshots at
    T = 1..8 in one launch, an FTLE field per snapshot) and early evaluation on a
    truncated ABC box (the field sampled on the closed box [0, 2pi]^3, 128^3 seeds,
    T = 4: tracers near the faces leave, their stencils are evaluated early)."""
    stream = torch.cuda.current_stream()
    L = 2 * math.pi
    fs = inputs.abc_frames(n=128, n_frames=33, dt_frame=0.5)
    g = inputs.periodic_seeds(3, (256, 256, 256), (L, L, L))
    frames = stage_frames(lcs, fs, LAYOUT_3D)
    ns = g.count
    steps = [50 * k for k in range(1, 9)]
    xs = torch.empty((8, 3, ns), dtype=torch.float32, device="cuda")
    done = torch.empty(ns, dtype=torch.int32, device="cuda")
    sig = torch.empty(ns, dtype=torch.float64, device="cuda")

    def timed(fn):
        fn()
        ms = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    def snap_all():
        lcs.lcs_advect_snapshots(frames, g, 0.0, 0.02, steps, xf=xs, steps_done=done,
                                 want_flags=False, stream=stream)
        for k in range(8):
            lcs.lcs_cg_ftle(g, xs[k], steps[k] * 0.02, ftle=sig, stream=stream)

    ms_snap = timed(snap_all)
    xf = torch.empty((3, ns), dtype=torch.float32, device="cuda")
    ms_one = timed(lambda: lcs.lcs_advect(frames, g, 0.0, 8.0, 0.02, xf=xf, want_cell=False,
                                          want_flags=False, stream=stream))
    del xs, xf, frames
    torch.cuda.empty_cache()
    ft = inputs.sample_field(inputs.abc_velocity, 3, (129, 129, 129), (0.0,) * 3, (L / 128,) * 3,
                             (False,) * 3, 0.0, 0.5, 17).astype(np.float32)
    frames = stage_frames(lcs, ft, LAYOUT_3D)
    gt = inputs.linspace_seeds(3, (128, 128, 128), (0.0,) * 3, (L,) * 3)
    nt = gt.count
    x1 = torch.empty((1, 3, nt), dtype=torch.float32, device="cuda")
    d1 = torch.empty(nt, dtype=torch.int32, device="cuda")
    lcs.lcs_advect_snapshots(frames, gt, 0.0, 0.02, [200], xf=x1, steps_done=d1, want_flags=False,
                             stream=stream)
    ws = torch.empty(lcs.lcs_ftle_early_workspace_bytes(gt), dtype=torch.uint8, device="cuda")
    lam = torch.empty(nt, dtype=torch.float64, device="cuda")
    se = torch.empty(nt, dtype=torch.float64, device="cuda")
    te = torch.empty(nt, dtype=torch.float64, device="cuda")
    ms_early = timed(lambda: lcs.lcs_ftle_early(frames, gt, 0.0, 0.02, 200, x1[0], d1, lam, se, te,
                                                ws, stream=stream))
    lcs.lcs_sync_status()
    early = int((te < 4.0 - 1e-12).sum().item())
    return {"workload": "abc_128cubed_seeds256cubed_8_snapshots", "frame_layout": LAYOUT_3D,
            "snapshot_steps": steps, "ms_8_snapshots_and_8_ftle_fields": ms_snap,
            "ms_single_lcs_advect_tiles": ms_one,
            "truncated_box": {"workload": "abc_closed_box_129cubed_seeds128cubed_T4",
                              "seeds": nt, "early_seeds": early, "ms_ftle_early": ms_early}}


def bench_surrogate(torch, lcs, keep, n_train=1 << 24, epochs=4):
    """Learned flow-map surrogate on the random-Fourier field: train on RK4
    displacements over tau = 0.5 (x0 uniform on the torus, t0 in {4, 4.5, ..,
    7.5}), compose 8 windows for the forward T = 4 FTLE of the 512x512x256
    seeds, check 1 % of each 16x16x8 tile against RK4 (tolerance 1e-3) and
    re-advect failing tiles with RK4.  Compared with plain RK4 (dt = 0.01) and
    with plain RK4 at coarser steps."""
    from paper_2209_13775_amd import surrogate as S
    frames, g, ref = keep["frames"], keep["seeds"], keep["ref_ftle"]
    T = 4.0
    cfg = S.SurrogateConfig(tau=0.5, n_windows=8, t0=4.0, dt=0.01, sigma_x=4.0, sigma_t=1.0)
    mlp = S.new_model(cfg)
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    e0, e1 = ev(), ev()
    e0.record(stream)
    xt, dx, _ = S.training_data(frames, cfg, n_train, seed=1)
    e1.record(stream)
    torch.cuda.synchronize()
    data_ms = e0.elapsed_time(e1)
    vxt, vdx, _ = S.training_data(frames, cfg, 1 << 16, seed=2)
    base = S.evaluate(mlp, vxt, vdx)
    log = S.train(mlp, xt, dx, epochs=epochs, batch=65536, lr=2e-3, val=(vxt, vdx))
    del xt, dx
    e0.record(stream)
    comp = lcs.lcs_surrogate_compose(mlp, g, cfg.t0, cfg.tau, cfg.n_windows, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    compose_ms = e0.elapsed_time(e1)
    flop = 2.0 * 230144 * g.count * cfg.n_windows    # 2 x multiply-adds of all layers
    del comp
    e0.record(stream)
    xf, flags, n_fail, err = S.surrogate_flowmap(mlp, frames, g, cfg, 1e-3, stream=stream)
    _, sig, _ = lcs.lcs_cg_ftle(g, xf, T, flags=flags, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    path_ms = e0.elapsed_time(e1)
    e = (sig - ref).abs()
    nt = lcs.lcs_check_tile_count(g)
    out = {"workload": "surrogate_on_random_fourier_256cubed_seeds512x512x256",
           "train_samples": n_train, "train_epochs": epochs, "train_steps": log.steps,
           "train_seconds": log.seconds, "data_ms": data_ms,
           "val_mse_before": base, "val_mse_after": log.val_loss,
           "compose_ms": compose_ms,
           "compose_tflops": flop / (compose_ms * 1e-3) / 1e12,
           "compose_mfma_frac": flop / (compose_ms * 1e-3) / 2.5e15,
           "check_tolerance": 1e-3, "fallback_tiles": int(n_fail.item()), "tiles": nt,
           "fallback_fraction": int(n_fail.item()) / nt,
           "tile_err_median": float(err.median().item()),
           "surrogate_path_ms": path_ms, "rk4_ms": keep["rk4_ms"],
           "speedup_vs_rk4": keep["rk4_ms"] / path_ms,
           "ftle_err_mean": float(e.mean().item()), "ftle_err_max": float(e.max().item())}
    del xf, flags, sig
    curve = []
    ws = torch.empty(lcs.lcs_advect_sorted_workspace_bytes(frames, g), dtype=torch.uint8,
                     device="cuda")
    for dtc in [0.02, 0.05, 0.1, 0.25]:
        e0.record(stream)
        seg = max(1, int(round(0.5 / dtc)))        # re-bundle every 0.5 time units
        xc, _, fc = lcs.lcs_advect_sorted(frames, g, cfg.t0, T, dtc, seg, workspace=ws,
                                          want_cell=False, stream=stream)
        _, sc, _ = lcs.lcs_cg_ftle(g, xc, T, flags=fc, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ec = (sc - ref).abs()
        curve.append({"dt": dtc, "ms": e0.elapsed_time(e1), "ftle_err_mean": float(ec.mean().item()),
                      "ftle_err_max": float(ec.max().item())})
        del xc, fc, sc
    out["coarse_rk4"] = curve
    out["coarse_rk4_strategy"] = "sorted, re-bundled every 0.5 time units"
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the hot path is measured on a single MI355X; "
              "--gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2209_13775_amd import inputs, lcs

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"bench: calibration copy of {args.calibrate_copy_mib} MiB done", file=sys.stderr,
              flush=True)
        del src, dst
    W = WORKLOAD
    L = 2 * math.pi
    fs = inputs.abc_frames(n=W["grid"], n_frames=W["frames"], dt_frame=W["dt_frame"])
    g = inputs.periodic_seeds(3, W["seeds"], (L, L, L))
    ns = g.count
    nsteps = int(round(W["T"] / W["dt"]))
    frames_soa = lcs.DeviceFrames(fs, device=dev)
    layout = args.layout
    global LAYOUT_3D
    LAYOUT_3D = layout
    frames = frames_soa if layout == "soa" else lcs.lcs_frames_interleave(frames_soa, layout)
    from paper_2209_13775_amd import autotune
    if args.strategy:
        tuned = {"choice": args.strategy, "ms": None}
    else:
        print("bench: autotuning the seed ordering", file=sys.stderr, flush=True)
        tuned = autotune.tune(frames, g, W["t0"], W["T"], W["dt"],
                              candidates=("tiles", "sorted:100"))
    choice = tuned["choice"]
    ws = None
    if choice != "tiles":
        ws = torch.empty(lcs.lcs_advect_sorted_workspace_bytes(frames, g), dtype=torch.uint8,
                         device=dev)
    xf = torch.empty((3, ns), dtype=torch.float32, device=dev)
    cell = torch.empty(ns, dtype=torch.int64, device=dev)
    flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    Cm = torch.empty((6, ns), dtype=torch.float64, device=dev)
    sfl = torch.empty(ns, dtype=torch.uint8, device=dev)
    lam = torch.empty(ns, dtype=torch.float64, device=dev)
    sig = torch.empty(ns, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        if layout != "soa":      # the step starts from the structure-of-arrays frames
            lcs.lcs_frames_interleave(frames_soa, layout, out=frames.u[0], stream=stream)
        autotune.run(choice, frames, g, W["t0"], W["T"], W["dt"], xf, cell, flags, ws, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        lcs.lcs_cg_tensor(g, xf, flags, Cm, sfl, stream=stream)
        lcs.lcs_ftle(3, Cm, W["T"], lam, sig, stream=stream)
        if ev is not None:
            ev[2].record(stream)

    print(f"bench: workload {W['name']}: {ns} seeds x {nsteps} steps; warmup {args.warmup}",
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lcs.lcs_sync_status()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
        print(f"bench: step {k + 1}/{args.steps} enqueued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    lcs.lcs_sync_status()
    adv_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    cgf_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    ms_per_step = wall * 1e3 / args.steps
    tracer_steps = ns * nsteps
    value = tracer_steps / (ms_per_step * 1e-3)
    achieved = BYTES_PER_STEP_3D * tracer_steps / (adv_ms * 1e-3) / 1e9
    nflag = int((flags != 0).sum().item())
    traffic = profiled_traffic(choice, layout)
    copy_gbs = measure_copy_gbs(torch, dev)
    seg_kernel = "advect_grid_kernel<3>" if choice == "tiles" else "rebundle_segment_kernel<3, 0>"
    out = {
        "metric": "tracer-RK4-steps/s (whole hot path: advect + C + FTLE), 1 GPU",
        "value": value,
        "unit": "tracer-RK4-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_detail": "advection and interpolation f32; gradient, C, lambda_max, FTLE f64",
        "data": "synthetic",
        "config": {"workload": W["name"], "field": "time-dependent ABC flow",
                   "grid": [W["grid"]] * 3, "frames": W["frames"], "seeds": list(W["seeds"]),
                   "t0": W["t0"], "T": W["T"], "dt": W["dt"], "rk4_steps": nsteps,
                   "frame_layout": layout},
        "advect_ms": adv_ms,
        "cg_ftle_ms": cgf_ms,
        "tracer_steps_per_s_advect_kernel": tracer_steps / (adv_ms * 1e-3),
        "ftle_points_per_s": ns / (cgf_ms * 1e-3),
        "flagged_tracers": nflag,
        "advect_strategy": choice,
        "autotune_ms": tuned["ms"],
        "roofline": {"kernel": ("advect_grid_kernel<3>" if choice == "tiles" else
                                "advection call: rebundle_segment_kernel<3, 0> x %d + re-bundling "
                                "sorts (+ frame interleave)"
                                % math.ceil(nsteps / int(choice.split(":")[1]))),
                     "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)",
                     "traffic_gbs": (traffic / (adv_ms * 1e-3) / 1e9) if traffic else None,
                     "traffic_frac": (traffic / (adv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "note": "achieved = algorithmic stencil bytes (768 B per tracer-RK4-step) per "
                             "second; they are served mostly from the per-tracer register cache, "
                             "L1, L2 and the MALL, so frac exceeds 1; traffic_gbs is the HBM rate "
                             "the counters measured",
                     "bytes_per_unit": BYTES_PER_STEP_3D, "unit_of_work": "3D tracer-RK4-step",
                     "units_per_launch": tracer_steps,
                     "measured_copy_gbs": copy_gbs,
                     "frac_of_measured_copy": achieved / copy_gbs,
                     "traffic_frac_of_measured_copy":
                         (traffic / (adv_ms * 1e-3) / 1e9 / copy_gbs) if traffic else None,
                     "l2_hit_rate": profiled_counter(seg_kernel, "l2_hit_rate"),
                     "ta_busy": profiled_counter(seg_kernel, "ta_busy"),
                     "td_busy": profiled_counter(seg_kernel, "td_busy"),
                     "counters_kernel": seg_kernel,
                     "binding_resource": "texture address / data units of the vector-memory "
                                         "path (ta_busy, td_busy: fraction of the kernel's "
                                         "cycles, rocprofv3 TA_TA_BUSY_sum / TD_TD_BUSY_sum)"},
        "cpu_baseline": None,
    }
    del frames, frames_soa, xf, cell, flags, Cm, sfl, lam, sig, ws
    if not args.no_extra:
        want = set(x.strip() for x in args.extras.split(",") if x.strip())
        if args.no_surrogate:
            want.discard("surrogate")
        extra = {}
        keep = {}
        torch.cuda.empty_cache()
        if "batched" in want:
            print("bench: batched double gyre windows", file=sys.stderr, flush=True)
            extra["batched"] = bench_batched(torch, lcs, inputs)
            torch.cuda.empty_cache()
        if "random_fourier" in want or "surrogate" in want:
            print("bench: random-Fourier forward/backward", file=sys.stderr, flush=True)
            extra["random_fourier"] = bench_random_fourier(torch, lcs, inputs, keep=keep)
            torch.cuda.empty_cache()
        if "surrogate" in want:
            print("bench: surrogate (train, compose, check, fallback)", file=sys.stderr, flush=True)
            extra["surrogate"] = bench_surrogate(torch, lcs, keep)
        keep.clear()
        torch.cuda.empty_cache()
        if "mesh" in want:
            print("bench: unstructured meshes", file=sys.stderr, flush=True)
            extra["mesh"] = bench_mesh(torch, lcs, inputs,
                                       cpu_sample=0 if args.no_cpu_baseline else 10000)
        if "ab" in want:
            print("bench: Adams-Bashforth", file=sys.stderr, flush=True)
            extra["adams_bashforth"] = bench_ab(torch, lcs, inputs)
            torch.cuda.empty_cache()
        if "aux" in want:
            print("bench: auxiliary points", file=sys.stderr, flush=True)
            extra["auxiliary_points"] = bench_aux(torch, lcs, inputs)
            torch.cuda.empty_cache()
        if "time_resolved" in want:
            print("bench: time-resolved and early FTLE", file=sys.stderr, flush=True)
            extra["time_resolved"] = bench_time_resolved(torch, lcs, inputs)
            torch.cuda.empty_cache()
        out["extra_workloads"] = extra
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(fs, g, W["t0"], W["T"], W["dt"], args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
