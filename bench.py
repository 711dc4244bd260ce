"""Benchmark of the LCS hot path on one MI355X.

One step = the whole hot path over one batch of synthetic input, on the
largest single-GPU workload: the divergence-free random-Fourier velocity field
(256^3 periodic grid, 65 FP32 frames at t = 0.125 f), 512 x 512 x 256 seeds,
forward and backward FTLE from t0 = 4 with |T| = 4, |dt| = 0.01 (400 RK4 steps
each way).  Per step: staging of the structure-of-arrays frames into the
time-paired records the kernels read, then for each direction lcs_advect
(re-bundled segments, autotuned) and lcs_cg_ftle (gradient, C, lambda_max and
the FTLE, FP64).

Prints one JSON line.  ``value`` is tracer-RK4-steps per second of the whole
step (FTLE points per second beside it); the roofline object covers the
dominant kernel (the re-bundled RK4 segment kernel), its launches timed with
HIP events on the stream they run on; the CPU baseline is the FP64 oracle on a
bounded sample of the same seeds (with their difference stencils) on the host
cores, and the same oracle run gives the error of each GPU result against
FP64.
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
# vector L1 data path: 128 B per clock per CU (the vL1D speed-of-light figure of
# AMD's profiler for this chip) x 256 CUs x 2.4 GHz peak engine clock
VL1D_PEAK_GBS = 128 * 256 * 2.4
BYTES_PER_STEP_3D = 768      # 4 evals x 8 corners x 2 frames x 3 comps x 4 B
N_CUS = 256
VMEM_FLOOR_CYCLES = 16       # CU cycles per wave load instruction, at least (measured)
WORKLOAD = dict(name="random_fourier_256cubed_65frames_seeds512x512x256_T4_forward_backward",
                grid=256, frames=65, dt_frame=0.125, seeds=(512, 512, 256), t0=4.0, T=4.0,
                dt=0.01)
ABC_WORKLOAD = dict(name="abc_128cubed_seeds256cubed", grid=128, frames=33, dt_frame=0.5,
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
                    help="skip the extra workloads (surrogate, ABC, batched windows, meshes, "
                         "multistep, auxiliary points, time-resolved)")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate workload")
    ap.add_argument("--layout", default="tpair", choices=("soa", "xyz", "xyzw", "tpair"),
                    help="frame layout the kernels read; with an interleaved layout the main "
                         "step converts the structure-of-arrays frames inside its timed region")
    ap.add_argument("--extras", default="surrogate,abc,batched,mesh,ab,aux,time_resolved",
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


def profiled_record(kernel, workload):
    """The committed rocprofv3 counter record of a kernel on a workload (HBM
    bytes per launch, busy fractions, hit rates), or None if there is none or
    the kernel sources changed since it was taken."""
    try:
        names = sorted(os.listdir(PROFILES))
    except OSError:
        return None
    for name in names:
        if not name.endswith(".md"):
            continue
        for line in open(os.path.join(PROFILES, name)).read().splitlines():
            if not line.startswith("{"):
                continue
            rec = json.loads(line)
            if rec.get("kernel") != kernel or rec.get("workload") != workload:
                continue
            if source_hash(rec["source_files"]) == rec["source_sha1"]:
                return rec
    return None


def roofline_record(kernel, avg_ms, launches, units_per_launch, workload,
                    bytes_per_unit=None, unit_of_work=None):
    """Roofline of an advection kernel: algorithmic stencil bytes per launch
    over its average launch duration (HIP events around each launch on its
    stream), against the vector L1 data path that binds these gathers, with the
    HBM traffic and busy fractions from the committed counter profile."""
    bpu = BYTES_PER_STEP_3D if bytes_per_unit is None else bytes_per_unit
    A = bpu * units_per_launch / (avg_ms * 1e-3) / 1e9
    prof = profiled_record(kernel, workload) or {}
    traffic = prof.get("traffic_bytes_per_launch")
    hbm = traffic / (avg_ms * 1e-3) / 1e9 if traffic else None
    # the data path's instruction floor: VMEM_FLOOR_CYCLES CU cycles per wave load
    # instruction times the profile's load instructions per wave-step, against
    # the measured CU cycles per wave-step (at the profile's mean clock)
    floor = None
    lpw, ghz = prof.get("vmem_loads_per_wave_step"), prof.get("mean_clock_ghz")
    if lpw and ghz:
        cyc = avg_ms * 1e-3 * ghz * 1e9 * N_CUS / (units_per_launch / 64.0)
        floor = {"frac": VMEM_FLOOR_CYCLES * lpw / cyc, "loads_per_wave_step": lpw,
                 "floor_cycles_per_wave_step": VMEM_FLOOR_CYCLES * lpw,
                 "measured_cycles_per_wave_step": cyc,
                 "basis": "a wave's 16-byte-per-lane load takes at least 16 CU cycles in the "
                          "texture data path (one per quad of lanes, inactive quads included)"}
    return {"kernel": kernel, "bound": "vl1d", "achieved": A, "peak": VL1D_PEAK_GBS,
            "unit": "GB/s", "frac": A / VL1D_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, each "
                            "scaled by the same counter on a plain copy of known size)",
            "bytes_per_unit": bpu,
            "unit_of_work": unit_of_work or ("3D tracer-RK4-step (4 evaluations x 8 corners x 2 "
                                             "frames x 3 components x 4 B of stencil data)"),
            "units_per_launch": units_per_launch, "launches_timed": launches,
            "avg_launch_ms": avg_ms,
            "timing": "HIP events recorded by the library around every launch of the kernel, "
                      "on the stream it runs on, over the timed region",
            "peak_basis": "vector L1 data path: 128 B per clock per CU x 256 CUs x 2.4 GHz",
            "hbm_gbs": hbm, "hbm_frac": hbm / HBM_PEAK_GBS if hbm else None,
            "algorithmic_bytes_over_hbm_peak": A / HBM_PEAK_GBS,
            "l2_hit_rate": prof.get("l2_hit_rate"), "l1_hit_rate": prof.get("l1_hit_rate"),
            "ta_busy": prof.get("ta_busy"), "td_busy": prof.get("td_busy"),
            "counters_workload": workload if prof else None,
            "vmem_instruction_floor": floor,
            "note": "the stencil gathers are served from the per-tracer register cache, L1 and "
                    "L2 (algorithmic_bytes_over_hbm_peak counts them as if none were): the "
                    "kernel's HBM traffic is hbm_frac of the peak, and the texture address / "
                    "data units of the vector-memory path are busy for most of its cycles "
                    "(ta_busy, td_busy), so the vector L1 data path is the roofline it is held to"}


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


def host_threads():
    """Threads the oracle uses: the CPU share of this process (its affinity
    set, capped by OMP_NUM_THREADS where the environment sets one), and the
    host's logical CPU count for the record."""
    try:
        share = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        share = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    n = min(share, int(env)) if env.isdigit() and int(env) > 0 else share
    return max(1, n), share, os.cpu_count()


def stencil_sample(g, m, seed):
    """m seed indices drawn without replacement (deterministic), the indices of
    their -/+ neighbours along each axis (wrapped on periodic axes, clamped
    otherwise) and the union of all of them."""
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(g.count, size=min(m, g.count), replace=False))
    c = g.coords_of(idx)
    nb_m, nb_p = [], []
    for b in range(g.dim):
        cm, cp = c.copy(), c.copy()
        if g.periodic[b]:
            cm[b] = (c[b] - 1) % g.n[b]
            cp[b] = (c[b] + 1) % g.n[b]
        else:
            cm[b] = np.maximum(c[b] - 1, 0)
            cp[b] = np.minimum(c[b] + 1, g.n[b] - 1)
        nb_m.append(g.index_of(cm))
        nb_p.append(g.index_of(cp))
    allidx = np.unique(np.concatenate([idx] + nb_m + nb_p))
    return idx, c, nb_m, nb_p, allidx


def err_stats(e):
    e = np.asarray(e, dtype=np.float64)
    return {"mean": float(e.mean()), "p99": float(np.quantile(e, 0.99)), "max": float(e.max()),
            "n": int(e.size)}


def fp64_errors(oracle, g, gpu, idx, c, nb_m, nb_p, allidx, xo, flo, T, L):
    """Error of each GPU result (positions, C, lambda_max, FTLE) against the
    FP64 oracle at the sampled seeds: the oracle's C comes from its own
    positions of each seed and its stencil."""
    pos = {int(k): p for p, k in enumerate(allidx)}
    nq = g.dim * (g.dim + 1) // 2
    Co = np.empty((nq, idx.size))
    bad = np.zeros(idx.size, dtype=bool)
    for q, s in enumerate(idx):
        ps = pos[int(s)]
        xm = [xo[:, pos[int(nb_m[b][q])]] for b in range(g.dim)]
        xp = [xo[:, pos[int(nb_p[b][q])]] for b in range(g.dim)]
        Co[:, q] = oracle.cg_point(g, c[:, q], xo[:, ps], xm, xp)
        used = [ps] + [pos[int(nb_m[b][q])] for b in range(g.dim)] + \
            [pos[int(nb_p[b][q])] for b in range(g.dim)]
        bad[q] = bool(np.any(flo[used]))
    lo, so = oracle.ftle(g.dim, Co, T)
    sel = np.array([pos[int(s)] for s in idx])
    ok = ~bad & (gpu["sflags"] == 0)
    ex = np.linalg.norm(gpu["xf"].astype(np.float64) - xo[:, sel], axis=0)
    # Frobenius norm of the packed symmetric difference (off-diagonals twice)
    w = np.array([1.0 if r == s_ else 2.0 for r in range(g.dim) for s_ in range(r, g.dim)])
    fro = lambda M: np.sqrt((w[:, None] * M * M).sum(axis=0))
    eC = fro(gpu["C"] - Co) / fro(Co)
    return {"seeds": int(idx.size), "clean_stencils": int(ok.sum()),
            "xf_abs": err_stats(ex), "xf_over_domain_length": err_stats(ex / L),
            "C_rel_frobenius": err_stats(eC[ok]),
            "lambda_max_rel": err_stats(np.abs(gpu["lam"][ok] - lo[ok]) / np.abs(lo[ok])),
            "ftle_abs": err_stats(np.abs(gpu["ftle"][ok] - so[ok])),
            "flags_equal": bool(np.array_equal(gpu["flags"], flo[sel]))}


def cpu_baseline(fs_host, g, t0, T, dt, target_s, gpu_at, L):
    """FP64 oracle on a bounded, deterministic sample of the seeds, each with
    its difference stencil, on the host cores: the rate in tracer-RK4-steps/s,
    and the error of the GPU's results at those seeds against it."""
    import oracle
    vel = oracle.Velocity(fs_host, keep_f32=True)
    threads, share, ncpu = host_threads()
    nsteps = int(round(T / dt))
    # calibrate on a small sample, then size the timed one to ~target_s
    _, _, _, _, cal = stencil_sample(g, 256, seed=1)
    t = time.perf_counter()
    oracle.advect_seeds(vel, g, t0, T, dt, idx=cal, threads=threads)
    el = max(time.perf_counter() - t, 1e-3)
    per_tracer = el / cal.size
    m = int(max(256, min(g.count // 8, target_s / per_tracer / 6.5)))
    idx, c, nb_m, nb_p, allidx = stencil_sample(g, m, seed=0)
    gpu = gpu_at(idx)
    t = time.perf_counter()
    xo, _, flo = oracle.advect_seeds(vel, g, t0, T, dt, idx=allidx, threads=threads)
    el = time.perf_counter() - t
    errs = fp64_errors(oracle, g, gpu, idx, c, nb_m, nb_p, allidx, xo, flo, T, L)
    # one thread as well, the serial baseline the paper quotes its speedups against
    m1 = max(64, int(2.0 / per_tracer / threads))
    idx1 = np.sort(np.random.default_rng(3).choice(g.count, size=m1, replace=False))
    t = time.perf_counter()
    oracle.advect_seeds(vel, g, t0, T, dt, idx=idx1, threads=1)
    el1 = time.perf_counter() - t
    return {"value": allidx.size * nsteps / el, "unit": "tracer-RK4-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{idx.size} seeds drawn from the 512x512x256 grid (seed 0) with their "
                      f"difference stencils ({allidx.size} tracers), forward T={T:g} "
                      f"({nsteps} RK4 steps), FP64, OpenMP on {threads} threads, {el:.1f} s",
            "host_cpu_share": share, "host_logical_cpus": ncpu,
            "threads_note": "the oracle uses every CPU of this process's share (its affinity "
                            "set, capped by OMP_NUM_THREADS where set)",
            "single_thread_value": m1 * nsteps / el1,
            "single_thread_sample": f"{m1} seeds, full T, one thread, {el1:.1f} s",
            "cpu_model": cpu_model(),
            "fp64_error": errs}


def precision_double_gyre(torch, lcs, inputs):
    """Error against FP64 on the full double-gyre workload (201 x 101 nodes, 21
    frames sampled in FP64, 256 x 128 seeds, T = 10, dt = 0.05): the mean
    trajectory error e_S(t) of the FP32 GPU run against the FP64 oracle every
    5 steps (the comparison of single- and double-precision trajectories), and
    the error of each final result (positions, C, lambda_max, FTLE).  The GPU
    reads the FP32 rounding of the frames; e_S against the oracle run on those
    same FP32 frames separates input rounding from arithmetic rounding."""
    import oracle
    fs = inputs.double_gyre_frames(nx=201, ny=101, n_frames=21)
    g = inputs.linspace_seeds(2, (256, 128), (0.0, 0.0), (2.0, 1.0))
    t0, T, dt = 0.0, 10.0, 0.05
    frames = lcs.DeviceFrames(fs)
    steps = list(range(5, 201, 5))
    xs, _, _ = lcs.lcs_advect_snapshots(frames, g, t0, dt, steps, want_flags=False,
                                        want_steps=False)
    xf, cell, flags = lcs.lcs_advect(frames, g, t0, T, dt)
    Cm, sfl = lcs.lcs_cg_tensor(g, xf, flags)
    lam, sig = lcs.lcs_ftle(2, Cm, T)
    lcs.lcs_sync_status()
    xs = xs.cpu().numpy()
    x0 = oracle.seed_points(g)
    curves = {}
    for name, f in (("fp64_frames", fs), ("fp32_frames", fs.astype(np.float32))):
        traj, tfl = oracle.advect_points_traj(oracle.Velocity(f), x0, t0, T, dt)
        ok = tfl == 0
        e = [float(np.linalg.norm(xs[k].astype(np.float64) - traj[s - 1], axis=0)[ok].mean())
             for k, s in enumerate(steps)]
        curves[name] = e
    vel = oracle.Velocity(fs)
    xo, _, flo = oracle.advect_seeds(vel, g, t0, T, dt)
    Co, so_fl = oracle.cg_tensor(g, xo, flo)
    lo, so = oracle.ftle(2, Co, T)
    ok = (so_fl == 0) & (sfl.cpu().numpy() == 0)
    gC = Cm.cpu().numpy()
    w = np.array([1.0, 2.0, 1.0])
    fro = lambda M: np.sqrt((w[:, None] * M * M).sum(axis=0))
    ex = np.linalg.norm(xf.cpu().numpy().astype(np.float64) - xo, axis=0)
    gl, gs = lam.cpu().numpy(), sig.cpu().numpy()
    return {"workload": "double_gyre_201x101_21frames_seeds256x128_T10",
            "e_S_steps": steps, "e_S_times": [t0 + s * dt for s in steps],
            "e_S_vs_fp64_oracle": curves["fp64_frames"],
            "e_S_vs_oracle_on_fp32_frames": curves["fp32_frames"],
            "domain_length": 2.0,
            "final": {"xf_abs": err_stats(ex), "xf_over_domain_length": err_stats(ex / 2.0),
                      "C_rel_frobenius": err_stats((fro(gC - Co) / fro(Co))[ok]),
                      "lambda_max_rel": err_stats((np.abs(gl - lo) / np.abs(lo))[ok]),
                      "ftle_abs": err_stats(np.abs(gs - so)[ok]),
                      "flags_equal": bool(np.array_equal(flags.cpu().numpy(), flo)),
                      "clean_stencils": int(ok.sum())}}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_batched(torch, lcs, inputs, reps=3, layout="tpair"):
    """Double gyre on 1025x513 nodes x 101 FP32 frames (t = 0.25 f), read as
    time-paired records; 64 windows (t0 ~ U[0,10], T from {5, 7.5, 10, 12.5,
    15}, default_rng(0)) of a 1024x512 seed grid, dt = 0.05, all in one
    graph-replayed persistent launch."""
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
           "roofline": roofline_record("advect_batched_kernel<2>", ms, len(times), steps,
                                       "double_gyre_batched_1025x513_64windows", 256,
                                       "2D tracer-RK4-step (4 evaluations x 4 corners x 2 frames "
                                       "x 2 components x 4 B)"),
           "graph": plan.stats()}
    plan.close()
    return out


def bench_abc(torch, lcs, inputs, reps=5):
    """Time-dependent ABC flow, 128^3 periodic grid, 33 FP32 frames, 256^3 seeds,
    t0 = 0, T = 8, dt = 0.02: staging + lcs_advect (autotuned) + lcs_cg_ftle."""
    from paper_2209_13775_amd import autotune
    W = ABC_WORKLOAD
    L = 2 * math.pi
    fs = inputs.abc_frames(n=W["grid"], n_frames=W["frames"], dt_frame=W["dt_frame"])
    g = inputs.periodic_seeds(3, W["seeds"], (L, L, L))
    ns = g.count
    nsteps = int(round(W["T"] / W["dt"]))
    soa = lcs.DeviceFrames(fs)
    frames = lcs.lcs_frames_interleave(soa, LAYOUT_3D)
    tuned = autotune.tune(frames, g, W["t0"], W["T"], W["dt"], candidates=("tiles", "sorted:100"))
    choice = tuned["choice"]
    ws = None if choice == "tiles" else torch.empty(
        lcs.lcs_advect_sorted_workspace_bytes(frames, g), dtype=torch.uint8, device="cuda")
    xf = torch.empty((3, ns), dtype=torch.float32, device="cuda")
    cell = torch.empty(ns, dtype=torch.int64, device="cuda")
    flags = torch.empty(ns, dtype=torch.uint8, device="cuda")
    lam = torch.empty(ns, dtype=torch.float64, device="cuda")
    sig = torch.empty(ns, dtype=torch.float64, device="cuda")
    sfl = torch.empty(ns, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        lcs.lcs_frames_interleave(soa, LAYOUT_3D, out=frames.u[0], stream=stream)
        autotune.run(choice, frames, g, W["t0"], W["T"], W["dt"], xf, cell, flags, ws,
                     stream=stream)
        if ev:
            ev[1].record(stream)
        lcs.lcs_cg_ftle(g, xf, W["T"], flags=flags, lambda_max=lam, ftle=sig, stencil_flags=sfl,
                        stream=stream)
        if ev:
            ev[2].record(stream)

    step()
    torch.cuda.synchronize()
    kernel = "advect_grid_kernel<3>" if choice == "tiles" else "rebundle_segment_kernel<3, 0>"
    lcs.lcs_timing_enable(True)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
    for k in range(reps):
        step(evs[k])
    torch.cuda.synchronize()
    launches, kms = lcs.lcs_timing_query(kernel)
    lcs.lcs_timing_enable(False)
    lcs.lcs_sync_status()
    tot = [e[0].elapsed_time(e[2]) for e in evs]
    adv = float(np.median([e[0].elapsed_time(e[1]) for e in evs]))
    cgf = float(np.median([e[1].elapsed_time(e[2]) for e in evs]))
    ms = float(np.median(tot))
    steps = ns * nsteps
    seg = nsteps if choice == "tiles" else int(choice.split(":")[1])
    out = {"workload": W["name"], "field": "time-dependent ABC flow", "frame_layout": LAYOUT_3D,
           "seeds": ns, "rk4_steps": nsteps, "advect_strategy": choice, "autotune_ms": tuned["ms"],
           "ms_per_step_median": ms, "advect_ms": adv, "cg_ftle_ms": cgf,
           "tracer_steps_per_s": steps / (ms * 1e-3), "ftle_points_per_s": ns / (cgf * 1e-3),
           "roofline": roofline_record(kernel, kms / max(launches, 1), launches,
                                       ns * seg, "abc_128cubed_seeds256cubed")}
    del frames, soa, ws, xf, cell, flags, lam, sig, sfl
    return out


# fused training step, per sample: forward reads inputs and targets (28 B) and writes the
# layer inputs h_0..h_3 (1792 B), gelu' of 4 layers (2048 B) and dy (12 B); backward reads
# gelu' and dy and writes dz of 4 layers (2048 B); weight gradients read h and dz
TRAIN_BYTES_PER_SAMPLE = (28 + 1792 + 2048 + 12) + (2048 + 12 + 2048) + (1792 + 2048)
TRAIN_FLOPS_PER_SAMPLE = 1.32e6   # forward 0.46 + backward-data 0.39 + weight gradients 0.46 MFLOP
MLP_PARAMS = 231171
MLP_BF16 = 458752

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
               "roofline": roofline_record("mesh_advect_grid_kernel<%d>" % dim, adv, reps, steps,
                                           name, bps, "%dD mesh tracer-RK4-step (cell maps, node "
                                           "ids and node values of the 4 evaluations)" % dim)}
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
    # training-step roofline: the step is bound by its activation traffic
    # (TRAIN_BYTES_PER_SAMPLE per sample plus the per-step partial sums and
    # Adam), not by the matrix cores
    step_s = log.seconds / max(log.steps, 1)
    nch = 65536 // 2048                               # weight-gradient chunks of 2048 samples
    step_bytes = TRAIN_BYTES_PER_SAMPLE * 65536 + (2 * nch * 4 + 6 * 4) * MLP_PARAMS + 2 * MLP_BF16
    prof = profiled_record("training step", "surrogate_training_batch65536") or {}
    traffic = prof.get("traffic_bytes_per_launch")
    train_roof = {"kernel": "training step (train_fwd + train_bwd + train_wgrad + train_update)",
                  "bound": "hbm", "achieved": step_bytes / step_s / 1e9, "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": step_bytes / step_s / 1e9 / HBM_PEAK_GBS,
                  "bytes_per_unit": step_bytes, "unit_of_work": "Adam step of 65,536 samples",
                  "avg_step_ms": step_s * 1e3, "traffic": traffic,
                  "hbm_gbs": traffic / step_s / 1e9 if traffic else None,
                  "hbm_frac": traffic / step_s / 1e9 / HBM_PEAK_GBS if traffic else None,
                  "bf16_tflops": TRAIN_FLOPS_PER_SAMPLE * 65536 / step_s / 1e12,
                  "mfma_frac": TRAIN_FLOPS_PER_SAMPLE * 65536 / step_s / 1e12 / 2500.0,
                  "note": "algorithmic bytes: inputs, the layer inputs and gelu' written and read "
                          "back, dz written and read back, chunk partials and Adam; an arithmetic "
                          "intensity of ~100 flop/B, below the 312 flop/B of 2.5 PFLOP/s / 8 TB/s"}
    flop = 2.0 * 230144 * g.count * cfg.n_windows    # 2 x multiply-adds of all layers
    lcs.lcs_timing_enable(True)
    e0.record(stream)
    comp = lcs.lcs_surrogate_compose(mlp, g, cfg.t0, cfg.tau, cfg.n_windows, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    compose_ms = e0.elapsed_time(e1)
    nl, kms = lcs.lcs_timing_query("compose_fused_kernel")
    lcs.lcs_timing_enable(False)
    del comp
    nt = lcs.lcs_check_tile_count(g)
    wsb = lcs.lcs_surrogate_flowmap_workspace_bytes(frames, g, 0.25)
    fws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    points = {}
    for name, tol in (("check_tol_1e-3", 1e-3), ("check_tol_1e-2", 1e-2),
                      ("composition_only", float("inf"))):
        e0.record(stream)
        xf, flags, nf, whole, err = lcs.lcs_surrogate_flowmap(
            mlp, frames, g, cfg.t0, cfg.tau, cfg.n_windows, tol, cfg.dt, whole_grid_fraction=0.25,
            workspace=fws, stream=stream)
        _, sig, _ = lcs.lcs_cg_ftle(g, xf, T, flags=flags, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        path_ms = e0.elapsed_time(e1)
        e = (sig - ref).abs()
        ev_ = err.float()
        points[name] = {"tolerance": tol, "fallback_tiles": nf, "tiles": nt,
                        "fallback_fraction": nf / nt, "whole_grid_fallback": whole,
                        "tile_err_median": float(ev_.median().item()),
                        "tile_err_min": float(ev_.min().item()),
                        "surrogate_path_ms": path_ms, "speedup_vs_rk4": keep["rk4_ms"] / path_ms,
                        "ftle_err_mean": float(e.mean().item()),
                        "ftle_err_p99": float(torch.quantile(e[::97].float(), 0.99).item()),
                        "ftle_err_max": float(e.max().item())}
        del xf, flags, sig, err, e
    del fws
    out = {"workload": "surrogate_on_random_fourier_256cubed_seeds512x512x256",
           "train_samples": n_train, "train_epochs": epochs, "train_steps": log.steps,
           "train_seconds": log.seconds, "data_ms": data_ms,
           "val_mse_before": base, "val_mse_after": log.val_loss,
           "val_rms_per_window": math.sqrt(log.val_loss),
           "sigma_x": cfg.sigma_x, "sigma_t": cfg.sigma_t,
           "train_roofline": train_roof,
           "compose_ms": compose_ms,
           "compose_tflops": flop / (compose_ms * 1e-3) / 1e12,
           "roofline": {"kernel": "compose_fused_kernel", "bound": "mfma",
                        "achieved": flop / (kms / max(nl, 1) * 1e-3) / 1e12 if nl else None,
                        "peak": 2500.0, "unit": "TFLOP/s",
                        "frac": flop / (kms / max(nl, 1) * 1e-3) / 1e12 / 2500.0 if nl else None,
                        "traffic": None, "flops_per_unit": 2 * 230144,
                        "unit_of_work": "point-window (BF16 MFMA, FP32 accumulation)",
                        "units_per_launch": g.count * cfg.n_windows, "avg_launch_ms":
                            kms / max(nl, 1)},
           "rk4_ms": keep["rk4_ms"], "rk4": "forward T = 4, dt = 0.01, re-bundled, + FTLE",
           "points": points}
    curve = []
    ws = keep["ws"]
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
    ok = [c for c in curve if c["ftle_err_mean"] <= 1e-2]
    out["fastest_rk4_within_1e-2"] = min(ok, key=lambda c: c["ms"]) if ok else None
    return out


def bench_surrogate_sweep(torch, lcs, inputs, sigmas=(1.0, 2.0, 4.0, 8.0), epochs_list=(4, 16, 64)):
    """Measured frontier of the learned surrogate (not run by default:
    --extras surrogate_sweep): for the random-Fourier and the ABC field, every
    frequency spread sigma_x x training length, trained on 2^24 RK4 pairs over
    tau = 0.5; on a 256 x 256 x 128 seed grid over T = 4 from t0 = 4: the
    validation RMS per window, the check-sample tile errors (fraction of tiles
    within 1e-2 and 1e-1) and the mean FTLE error of the composition alone
    against plain RK4 at dt = 0.01."""
    from paper_2209_13775_amd import surrogate as S
    L = 2 * math.pi
    out = []
    ev = lambda: torch.cuda.Event(enable_timing=True)
    for field in ("random_fourier", "abc"):
        if field == "random_fourier":
            fs = inputs.random_fourier_frames(n=256, n_frames=65, dt_frame=0.125, device="cuda")
            soa = lcs.DeviceFrames(fs, tensors=fs.u)
            speed = 1.0
        else:
            fs = inputs.abc_frames(n=128, n_frames=33, dt_frame=0.5)
            soa = lcs.DeviceFrames(fs)
            speed = math.sqrt(6.0)
        frames = lcs.lcs_frames_interleave(soa, "tpair")
        del soa
        g = inputs.SeedGrid(3, (256, 256, 128), (0.0,) * 3, (L / 256, L / 256, L / 128), (True,) * 3)
        T, dt = 4.0, 0.01
        e0, e1 = ev(), ev()
        e0.record()
        ref, _, rfl = lcs.lcs_advect_sorted(frames, g, 4.0, T, dt, 100, want_cell=False)
        _, rsig, _ = lcs.lcs_cg_ftle(g, ref, T, flags=rfl)
        e1.record()
        torch.cuda.synchronize()
        rk4_ms = e0.elapsed_time(e1)
        for sx in sigmas:
            cfg = S.SurrogateConfig(tau=0.5, n_windows=8, t0=4.0, dt=dt, sigma_x=sx, sigma_t=1.0,
                                    speed_scale=speed)
            xt, dx, _ = S.training_data(frames, cfg, 1 << 24, seed=1)
            vxt, vdx, _ = S.training_data(frames, cfg, 1 << 16, seed=2)
            for ep in epochs_list:
                mlp = S.new_model(cfg)
                log = S.train(mlp, xt, dx, epochs=ep, batch=65536, lr=2e-3, val=(vxt, vdx))
                e0.record()
                xf, flags, _, _, err = lcs.lcs_surrogate_flowmap(mlp, frames, g, 4.0, 0.5, 8,
                                                                 float("inf"), dt)
                e1.record()
                torch.cuda.synchronize()
                _, sig, _ = lcs.lcs_cg_ftle(g, xf, T, flags=flags)
                te = err.float()
                out.append({"field": field, "sigma_x": sx, "epochs": ep, "steps": log.steps,
                            "train_s": log.seconds, "val_rms_per_window": math.sqrt(log.val_loss),
                            "tile_err_median": float(te.median().item()),
                            "tiles_within_1e-3": float((te <= 1e-3).float().mean().item()),
                            "tiles_within_1e-2": float((te <= 1e-2).float().mean().item()),
                            "tiles_within_1e-1": float((te <= 1e-1).float().mean().item()),
                            "ftle_err_mean_composition": float((sig - rsig).abs().mean().item()),
                            "compose_and_check_ms": e0.elapsed_time(e1), "rk4_ms": rk4_ms})
                print(f"bench: surrogate sweep {out[-1]}", file=sys.stderr, flush=True)
                del mlp, xf, flags, err, sig
            del xt, dx, vxt, vdx
            torch.cuda.empty_cache()
        del frames, fs, ref, rsig
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the hot path is measured on a single MI355X; "
              "--gpus above 1 is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2209_13775_amd import autotune, inputs, lcs

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
    global LAYOUT_3D
    LAYOUT_3D = args.layout
    W = WORKLOAD
    L = 2 * math.pi
    print("bench: generating the random-Fourier field", file=sys.stderr, flush=True)
    t = time.perf_counter()
    fs = inputs.random_fourier_frames(n=W["grid"], n_frames=W["frames"], dt_frame=W["dt_frame"],
                                      device=dev)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t
    g = inputs.SeedGrid(3, W["seeds"], (0.0, 0.0, 0.0), tuple(L / k for k in W["seeds"]),
                        (True, True, True))
    ns = g.count
    nsteps = int(round(W["T"] / W["dt"]))
    frames_soa = lcs.DeviceFrames(fs, tensors=fs.u)
    layout = args.layout
    frames = frames_soa if layout == "soa" else lcs.lcs_frames_interleave(frames_soa, layout)
    if args.strategy:
        tuned = {"choice": args.strategy, "ms": None}
    else:
        print("bench: autotuning the seed ordering", file=sys.stderr, flush=True)
        tuned = autotune.tune(frames, g, W["t0"], W["T"], W["dt"],
                              candidates=("sorted:100", "sorted:50", "sorted:25"))
    choice = tuned["choice"]
    ws = None
    if choice != "tiles":
        ws = torch.empty(lcs.lcs_advect_sorted_workspace_bytes(frames, g), dtype=torch.uint8,
                         device=dev)
    xf = torch.empty((3, ns), dtype=torch.float32, device=dev)
    cell = torch.empty(ns, dtype=torch.int64, device=dev)
    flags = torch.empty(ns, dtype=torch.uint8, device=dev)
    dirs = [(W["T"], W["dt"]), (-W["T"], -W["dt"])]
    lam = [torch.empty(ns, dtype=torch.float64, device=dev) for _ in dirs]
    sig = [torch.empty(ns, dtype=torch.float64, device=dev) for _ in dirs]
    sfl = [torch.empty(ns, dtype=torch.uint8, device=dev) for _ in dirs]
    stream = torch.cuda.current_stream()

    def step(ev=None):
        # ev: 6 events -- start, staged, forward advected, forward FTLE,
        # backward advected, backward FTLE
        if ev is not None:
            ev[0].record(stream)
        if layout != "soa":      # the step starts from the structure-of-arrays frames
            lcs.lcs_frames_interleave(frames_soa, layout, out=frames.u[0], stream=stream)
        if ev is not None:
            ev[1].record(stream)
        for d, (T, dt) in enumerate(dirs):
            autotune.run(choice, frames, g, W["t0"], T, dt, xf, cell, flags, ws, stream=stream)
            if ev is not None:
                ev[2 + 2 * d].record(stream)
            lcs.lcs_cg_ftle(g, xf, T, flags=flags, lambda_max=lam[d], ftle=sig[d],
                            stencil_flags=sfl[d], stream=stream)
            if ev is not None:
                ev[3 + 2 * d].record(stream)

    print(f"bench: workload {W['name']}: {ns} seeds x {nsteps} steps x 2 directions; "
          f"warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lcs.lcs_sync_status()
    seg_kernel = "advect_grid_kernel<3>" if choice == "tiles" else "rebundle_segment_kernel<3, 0>"
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(args.steps)]
    lcs.lcs_timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
        print(f"bench: step {k + 1}/{args.steps} enqueued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    launches, kms = lcs.lcs_timing_query(seg_kernel)
    cg_launches, cg_ms = lcs.lcs_timing_query("cg_kernel<3, true>")
    lcs.lcs_timing_enable(False)
    lcs.lcs_sync_status()
    el = lambda a, b: float(np.median([e[a].elapsed_time(e[b]) for e in evs]))
    stage_ms = el(0, 1)
    adv_ms = el(1, 2) + el(3, 4)
    cgf_ms = el(2, 3) + el(4, 5)
    ms_per_step = wall * 1e3 / args.steps
    tracer_steps = 2 * ns * nsteps
    value = tracer_steps / (ms_per_step * 1e-3)
    seg = nsteps if choice == "tiles" else int(choice.split(":")[1])
    avg_launch = kms / max(launches, 1)
    nflag = int((flags != 0).sum().item())
    copy_gbs = measure_copy_gbs(torch, dev)
    roof = roofline_record(seg_kernel, avg_launch, launches, ns * seg, W["name"])
    roof["measured_copy_gbs"] = copy_gbs
    roof["cg_ftle_kernel"] = {"kernel": "cg_kernel<3, true>", "launches_timed": cg_launches,
                              "avg_launch_ms": cg_ms / max(cg_launches, 1),
                              "compulsory_bytes_per_point": 29,
                              "hbm_gbs_compulsory": 29 * ns / (cg_ms / max(cg_launches, 1) * 1e-3) / 1e9,
                              "note": "reads 12 B of xf and 1 B of flags, writes 8 B FTLE + 8 B "
                                      "lambda_max per point (stencil flags not asked for)"}
    out = {
        "metric": "tracer-RK4-steps/s (whole hot path: stage + advect + C + FTLE, forward and "
                  "backward), 1 GPU",
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
        "dtype_detail": "advection and interpolation f32 (two-float positions); gradient, C, "
                        "lambda_max, FTLE f64",
        "data": "synthetic",
        "config": {"workload": W["name"],
                   "field": "divergence-free random-Fourier velocity, |k| <= 32, E(k) ~ k^-5/3, "
                            "OU time decorrelation 2, RMS speed 1 (seed 1)",
                   "grid": [W["grid"]] * 3, "frames": W["frames"], "dt_frame": W["dt_frame"],
                   "seeds": list(W["seeds"]), "t0": W["t0"], "T": [W["T"], -W["T"]],
                   "dt": [W["dt"], -W["dt"]], "rk4_steps_per_direction": nsteps,
                   "frame_layout": layout},
        "ftle_points_per_s": 2 * ns / (cgf_ms * 1e-3),
        "stage_ms": stage_ms, "advect_ms": adv_ms, "cg_ftle_ms": cgf_ms,
        "tracer_steps_per_s_advect": tracer_steps / (adv_ms * 1e-3),
        "field_generation_s": gen_s,
        "flagged_tracers_backward": nflag,
        "mean_ftle": [float(sig[0].mean().item()), float(sig[1].mean().item())],
        "advect_strategy": choice,
        "autotune_ms": tuned["ms"],
        "roofline": roof,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on a sample (forward)", file=sys.stderr, flush=True)
        T, dt = dirs[0]
        autotune.run(choice, frames, g, W["t0"], T, dt, xf, cell, flags, ws, stream=stream)
        lcs.lcs_cg_ftle(g, xf, T, flags=flags, lambda_max=lam[0], ftle=sig[0],
                        stencil_flags=sfl[0], stream=stream)
        torch.cuda.synchronize()

        def gpu_at(idx):
            it = torch.from_numpy(idx).to(dev)
            Cs = lcs.lcs_cg_tensor(g, xf, flags, want_stencil=False)[0][:, it]
            return {"xf": xf[:, it].cpu().numpy(), "C": Cs.cpu().numpy(),
                    "lam": lam[0][it].cpu().numpy(), "ftle": sig[0][it].cpu().numpy(),
                    "flags": flags[it].cpu().numpy(), "sflags": sfl[0][it].cpu().numpy()}

        f0 = int(round((W["t0"] - fs.t_first) / fs.dt_frame))
        host = inputs.FrameSet(3, fs.n, fs.origin, fs.spacing, fs.periodic, W["t0"], fs.dt_frame,
                               [u[f0:].cpu().numpy() for u in fs.u])
        out["cpu_baseline"] = cpu_baseline(host, g, W["t0"], T, dt, args.cpu_seconds, gpu_at, L)
        del host
        print("bench: double-gyre precision (e_S curve, FP64 errors)", file=sys.stderr, flush=True)
        out["cpu_baseline"]["precision_double_gyre"] = precision_double_gyre(torch, lcs, inputs)
    keep = {"fs": fs, "frames": frames, "seeds": g, "ref_ftle": sig[0], "ws": ws,
            "rk4_ms": el(1, 3)}
    del frames_soa, xf, cell, flags, lam, sfl
    if not args.no_extra:
        want = set(x.strip() for x in args.extras.split(",") if x.strip())
        if args.no_surrogate:
            want.discard("surrogate")
        extra = {}
        if "surrogate" in want:
            print("bench: surrogate (train, compose, check, fallback)", file=sys.stderr, flush=True)
            extra["surrogate"] = bench_surrogate(torch, lcs, keep)
        keep.clear()
        del fs, sig
        torch.cuda.empty_cache()
        if "abc" in want:
            print("bench: ABC 128^3 workload", file=sys.stderr, flush=True)
            extra["abc"] = bench_abc(torch, lcs, inputs)
            torch.cuda.empty_cache()
        if "batched" in want:
            print("bench: batched double gyre windows", file=sys.stderr, flush=True)
            extra["batched"] = bench_batched(torch, lcs, inputs)
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
        if "surrogate_sweep" in want:
            print("bench: surrogate frontier sweep", file=sys.stderr, flush=True)
            extra["surrogate_sweep"] = bench_surrogate_sweep(torch, lcs, inputs)
            torch.cuda.empty_cache()
        if "time_resolved" in want:
            print("bench: time-resolved and early FTLE", file=sys.stderr, flush=True)
            extra["time_resolved"] = bench_time_resolved(torch, lcs, inputs)
            torch.cuda.empty_cache()
        out["extra_workloads"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
