"""Host-side logic of bench.py, on the CPU: the one-GPU guard, the source
digest that marks recorded counters as stale, and the oracle's CPU baseline
record on a small sample."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _tree(tmp_path, files):
    for name, text in files.items():
        (tmp_path / name).write_text(text)
    return str(tmp_path)


def test_source_digest_follows_included_headers(tmp_path):
    d = _tree(tmp_path, {"k.hip": '#include "a.h"\nkernel\n', "a.h": '#include "b.h"\n',
                         "b.h": "x\n", "other.h": "y\n"})
    h0 = bench.source_digest("k.hip", d)
    (tmp_path / "other.h").write_text("z\n")           # not included: no change
    assert bench.source_digest("k.hip", d) == h0
    (tmp_path / "b.h").write_text("x2\n")              # included through a.h
    h1 = bench.source_digest("k.hip", d)
    assert h1 != h0
    (tmp_path / "k.hip").write_text('#include "a.h"\nkernel2\n')
    assert bench.source_digest("k.hip", d) not in (h0, h1)


def test_source_digest_ignores_comments(tmp_path):
    d = _tree(tmp_path, {"k.hip": '#include "a.h"\nint k; // note\n', "a.h": "int a;\n"})
    h0 = bench.source_digest("k.hip", d)
    (tmp_path / "a.h").write_text("/* a header */\nint   a;  // the same code\n")
    assert bench.source_digest("k.hip", d) == h0
    (tmp_path / "a.h").write_text('const char* s = "// not a comment";\nint a;\n')
    assert bench.source_digest("k.hip", d) != h0


def test_traffic_is_null_once_the_source_changes(tmp_path):
    d = _tree(tmp_path, {"k.hip": '#include "a.h"\n', "a.h": "x\n"})
    rec = tmp_path / "traffic.json"
    rec.write_text(json.dumps({"k_x": {"bytes_per_launch": 123,
                                       "source_sha": bench.source_digest("k.hip", d)}}))
    assert bench.traffic_for("k.hip", "k_x", str(rec), d) == 123
    assert bench.traffic_for("k.hip", "k_missing", str(rec), d) is None
    (tmp_path / "a.h").write_text("x changed\n")
    assert bench.traffic_for("k.hip", "k_x", str(rec), d) is None


def test_committed_traffic_record_names_every_kernel():
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as fh:
        rec = json.load(fh)
    for key in ("k_direct_f64", "k_tree_J10", "k_adjoint", "k_grad_partial"):
        assert rec[key]["bytes_per_launch"] > 0 and len(rec[key]["source_sha"]) == 16


def test_valu_count_is_null_once_the_source_changes(tmp_path):
    d = _tree(tmp_path, {"k.hip": '#include "a.h"\n', "a.h": "x\n"})
    rec = tmp_path / "valu.json"
    rec.write_text(json.dumps({"k_x": {"valu_wave_instructions": 4.5e9,
                                       "source_sha": bench.source_digest("k.hip", d)}}))
    assert bench.valu_count_for("k.hip", "k_x", str(rec), d) == 4.5e9
    assert bench.valu_count_for("k.hip", "k_missing", str(rec), d) is None
    (tmp_path / "a.h").write_text("x changed\n")
    assert bench.valu_count_for("k.hip", "k_x", str(rec), d) is None


def test_committed_valu_record_classes_add_up():
    with open(os.path.join(ROOT, "profiles", "valu_issue.json")) as fh:
        rec = json.load(fh)
    for key in ("k_direct_f64", "k_tree_J10", "k_adjoint", "k_grad_partial", "k_direct_f32c"):
        r = rec[key]
        parts = sum(r[c] for c in ("f64", "f32", "trans_f32", "cvt", "int32", "int64", "other"))
        assert abs(parts - r["valu_wave_instructions"]) <= 1e-6 * r["valu_wave_instructions"]
        assert len(r["source_sha"]) == 16


def test_cpu_baseline_record_on_a_small_sample():
    b = bench.cpu_baseline(64)
    assert b["kind"] == "oracle" and b["unit"] == bench.UNIT
    assert 1 <= b["cores"] <= bench.CPU_SHARE
    assert b["value"] > 0 and b["cpu_seconds"] > 0
    assert "64 seeded rows" in b["sample"]


def test_precision_errors_of_a_known_difference():
    """E_max over the stated scale and E_rms over the reference norm, with the
    low-precision result widened before the difference."""
    import numpy as np
    import torch
    ref = torch.tensor([3.0 + 4.0j, 0.0, 1.0j], dtype=torch.complex128)
    low = (ref + torch.tensor([0.0, 0.5, -0.25j], dtype=torch.complex128)).to(torch.complex64)
    e = bench.precision_errors(low, ref, scale=10.0)
    assert e["E_max_vs_fp64"] == 0.05
    want = float(np.sqrt(0.5 ** 2 + 0.25 ** 2) / np.sqrt(25.0 + 1.0))
    assert abs(e["E_rms_vs_fp64"] - want) <= 1e-3 * want
    assert bench.precision_errors(ref.to(torch.complex64), ref, 1.0)["E_max_vs_fp64"] == 0.0
