"""Host logic of bench.py (no GPU): the one-GPU guard, the kernel-source hash
that keys committed profiles, and the rule that a profile figure is reported
only while its kernel sources are unchanged."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_source_hash_ignores_comments_and_blank_lines(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    a.write_text("int f(int x)\n{\n    return x + 1;\n}\n")
    b.write_text("// header comment\n\nint f(int x)   // trailing\n{\n  /* block\n comment */\n"
                 "    return x + 1;\n\n}\n")
    assert bench.source_hash([str(a)]) == bench.source_hash([str(b)])
    b.write_text("int f(int x)\n{\n    return x + 2;\n}\n")
    assert bench.source_hash([str(a)]) != bench.source_hash([str(b)])


@pytest.fixture
def fake_profiles(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("void k() {}\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    return src, prof


def _write(prof, recs):
    lines = ["# summary", "```"] + [json.dumps(r) for r in recs] + ["```", ""]
    (prof / "k.md").write_text("\n".join(lines))


def test_profile_figure_reported_only_for_unchanged_sources(fake_profiles):
    src, prof = fake_profiles
    h = bench.source_hash([str(src)])
    _write(prof, [
        {"kernel": "k<3>", "workload": "w1", "l2_hit_rate": 0.5, "td_busy": 0.9,
         "traffic_bytes_per_launch": 123.0, "source_files": [str(src)], "source_sha1": h},
        {"kernel": "k<3>", "workload": "w2", "l2_hit_rate": 0.7, "source_files": [str(src)],
         "source_sha1": h},
    ])
    assert bench.profiled_record("k<3>", "w1")["l2_hit_rate"] == 0.5
    assert bench.profiled_record("k<3>", "w1")["traffic_bytes_per_launch"] == 123.0
    assert bench.profiled_record("k<3>", "w2")["l2_hit_rate"] == 0.7
    assert bench.profiled_record("k<3>", "w3") is None
    assert bench.profiled_record("other<3>", "w1") is None
    r = bench.roofline_record("k<3>", 10.0, 4, 1000, "w1")
    assert r["traffic"] == 123.0 and r["td_busy"] == 0.9 and r["ta_busy"] is None
    assert abs(r["achieved"] - 768 * 1000 / 1e-2 / 1e9) < 1e-9
    assert abs(r["frac"] - r["achieved"] / bench.VL1D_PEAK_GBS) < 1e-15
    assert abs(r["hbm_gbs"] - 123.0 / 1e-2 / 1e9) < 1e-12
    src.write_text("void k() { int changed = 1; }\n")
    assert bench.profiled_record("k<3>", "w1") is None
    r = bench.roofline_record("k<3>", 10.0, 4, 1000, "w1")
    assert r["traffic"] is None and r["hbm_gbs"] is None


def test_stencil_sample_neighbours():
    from paper_2209_13775_amd import inputs
    g = inputs.SeedGrid(3, (8, 6, 5), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (True, False, True))
    idx, c, nm, npl, allidx = bench.stencil_sample(g, 50, seed=0)
    assert idx.size == 50 and np.all(np.diff(idx) > 0)
    for q, s in enumerate(idx):
        i, j, k = g.coords_of(np.array([s]))[:, 0]
        assert nm[0][q] == g.index_of(np.array([[(i - 1) % 8], [j], [k]]))[0]
        assert npl[1][q] == g.index_of(np.array([[i], [min(j + 1, 5)], [k]]))[0]
        assert nm[2][q] == g.index_of(np.array([[i], [j], [(k - 1) % 5]]))[0]
    assert set(idx) <= set(allidx) and all(set(a) <= set(allidx) for a in nm + npl)


def test_committed_profiles_carry_their_source_hashes():
    names = [n for n in os.listdir(os.path.join(ROOT, "profiles")) if n.endswith(".md")]
    assert names
    n_recs = 0
    for n in names:
        recs = [json.loads(line) for line in open(os.path.join(ROOT, "profiles", n))
                if line.startswith("{")]
        n_recs += len(recs)
        for r in recs:
            assert r["source_files"] and len(r["source_sha1"]) == 16, n
            for f in r["source_files"]:
                assert os.path.exists(os.path.join(ROOT, f)), (n, f)
    assert n_recs > 0


def test_fp64_error_table_is_zero_for_the_oracle_itself():
    # the bench's error table, fed the oracle's own results as the "GPU" side,
    # must report zero error (it recomputes C from the stencil positions)
    import oracle
    from paper_2209_13775_amd import inputs
    fs = inputs.abc_frames(n=16, n_frames=5, dt_frame=0.5, dtype=np.float64)
    L = 2 * np.pi
    g = inputs.periodic_seeds(3, (12, 10, 8), (L, L, L))
    vel = oracle.Velocity(fs)
    xo_all, _, fl_all = oracle.advect_seeds(vel, g, 0.0, 1.0, 0.05)
    Cm, sfl = oracle.cg_tensor(g, xo_all, fl_all)
    lam, sig = oracle.ftle(3, Cm, 1.0)
    idx, c, nm, npl, allidx = bench.stencil_sample(g, 40, seed=0)
    gpu = {"xf": xo_all[:, idx].astype(np.float32).astype(np.float64), "C": Cm[:, idx],
           "lam": lam[idx], "ftle": sig[idx], "flags": fl_all[idx], "sflags": sfl[idx]}
    gpu["xf"] = xo_all[:, idx]
    errs = bench.fp64_errors(oracle, g, gpu, idx, c, nm, npl, allidx, xo_all[:, allidx],
                             fl_all[allidx], 1.0, L)
    assert errs["clean_stencils"] == 40 and errs["flags_equal"]
    for k in ("xf_abs", "C_rel_frobenius", "lambda_max_rel", "ftle_abs"):
        assert errs[k]["max"] <= 1e-14, (k, errs[k])


def test_committed_profile_records_match_the_kernel_sources():
    # every machine-readable counter record under profiles/ was taken on the
    # kernel sources as they stand (comments aside): a kernel change must come
    # with regenerated profiles, or the bench would drop their figures
    import json
    recs = []
    for name in sorted(os.listdir(bench.PROFILES)):
        if name.endswith(".md"):
            for line in open(os.path.join(bench.PROFILES, name)).read().splitlines():
                if line.startswith("{"):
                    recs.append((name, json.loads(line)))
    assert {r["kernel"] for _, r in recs} >= {"rebundle_segment_kernel<3, 0>", "training step"}
    for name, r in recs:
        assert bench.source_hash(r["source_files"]) == r["source_sha1"], (name, r["kernel"])
