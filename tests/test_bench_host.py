"""Host logic of bench.py (no GPU): the one-GPU guard, the kernel-source hash
that keys committed profiles, and the rule that a profile figure is reported
only while its kernel sources are unchanged."""
import json
import os
import subprocess
import sys

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
        {"kernel": "k<3>", "l2_hit_rate": 0.5, "td_busy": 0.9, "source_files": [str(src)],
         "source_sha1": h},
        {"kernel": "advection call (sorted:100)", "strategy": "sorted:100", "layout": "tpair",
         "traffic_bytes_per_launch": 123.0, "source_files": [str(src)], "source_sha1": h},
    ])
    assert bench.profiled_counter("k<3>", "l2_hit_rate") == 0.5
    assert bench.profiled_counter("k<3>", "td_busy") == 0.9
    assert bench.profiled_counter("k<3>", "ta_busy") is None
    assert bench.profiled_counter("other<3>", "l2_hit_rate") is None
    assert bench.profiled_traffic("sorted:100", "tpair") == 123.0
    assert bench.profiled_traffic("sorted:100", "soa") is None
    assert bench.profiled_traffic("tiles", "tpair") is None
    src.write_text("void k() { int changed = 1; }\n")
    assert bench.profiled_counter("k<3>", "l2_hit_rate") is None
    assert bench.profiled_traffic("sorted:100", "tpair") is None


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
