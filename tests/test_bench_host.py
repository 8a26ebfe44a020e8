"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic byte
model, the choice of the dominant kernel for the roofline, and the source
hash check on the committed counter figures."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_model_bytes_per_particle():
    n, nb = 1000, 100.0
    m64 = bench.kernel_model(n, nb * n, 0.0, 0)
    m32 = bench.kernel_model(n, nb * n, 0.0, 1)
    # own arrays once, list entries 4 B each
    assert m64["find_neighbors"][0] == (40 + 4 * nb) * n
    assert m64["density"][0] == (52 + 4 * nb) * n
    assert m64["momentum_energy"][0] == (88 + 44 + 4 * nb) * n
    # the FP32-pair form moves its FP32 field copies, 20 B less per particle
    assert m64["momentum_energy"][0] - m32["momentum_energy"][0] == 20 * n
    # the step: 952 B of own arrays plus the list written once and read twice
    step = sum(v[0] for v in m64.values()) / n
    assert step == 952 + 3 * 4 * nb


def _run(kernel_ms, per_call=None, pairs=1.0e8, n=1_000_000):
    per_call = per_call or {c: 0.1 for c in bench.CALLS}
    return {"kernel_ms": {k: {"avg_ms": v, "launches": 10} for k, v in kernel_ms.items()},
            "per_call_ms": per_call, "pairs_per_step": pairs, "candidates": 0.0}


def test_roofline_takes_the_dominant_kernel_not_the_call():
    # momentum's call is longer (it packs records first), the search kernel longer
    per_call = {c: 0.05 for c in bench.CALLS}
    per_call.update(find_neighbors=0.76, momentum_energy=0.80)
    r = _run({"find_neighbors_kernel": 0.74, "fallback_kernel": 0.006,
              "density_kernel": 0.43, "momentum_kernel": 0.71}, per_call)
    out = bench.roofline(1_000_000, r, 0)
    assert out["kernel"] == "find_neighbors_kernel" and out["call"] == "find_neighbors"
    b = bench.kernel_model(1_000_000, 1.0e8, 0.0, 0)["find_neighbors"][0]
    assert out["achieved"] == pytest.approx(b / 0.74e-3 / 1e9, rel=1e-3)
    assert out["frac"] == pytest.approx(out["achieved"] / bench.HBM_PEAK_GBS, abs=1e-4)
    assert out["bound"] == "hbm" and out["unit"] == "GB/s"


def test_roofline_sums_a_calls_kernels_below_95_percent():
    # the Evrard search: the second kernel carries most of the call
    r = _run({"find_neighbors_kernel": 0.8, "fallback_kernel": 2.2,
              "density_kernel": 0.45, "momentum_kernel": 0.8})
    out = bench.roofline(1_000_000, r, 0)
    assert out["kernel"] == "fallback_kernel+find_neighbors_kernel"
    assert out["ms_per_launch"] == pytest.approx(3.0)
    assert out["traffic"] is None and out["valu_issue_frac"] is None


def test_recorded_counters_follow_the_source_hash(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    (tmp_path / "profiles").mkdir()
    prof = tmp_path / "profiles" / "x_kernel_w_counters.md"
    prof.write_text(f"traffic_bytes_per_launch: 1.5e+09\nvalu_insts_per_launch: 2.0e+08\n"
                    f"source_sha256: {sha} k.hip\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_counters("x_kernel", "w") == {"traffic": 1.5e9, "valu_insts": 2.0e8}
    src.write_text("kernel source, changed\n")
    assert bench.recorded_counters("x_kernel", "w") == {}
    assert bench.recorded_counters("other_kernel", "w") == {}


def test_committed_counters_name_existing_sources():
    """Every committed counter summary names a source file of this tree."""
    import re
    pdir = os.path.join(ROOT, "profiles")
    files = [f for f in os.listdir(pdir) if f.endswith("_counters.md")]
    assert files
    for f in files:
        m = re.search(r"source_sha256:\s*([0-9a-f]{64})\s+(\S+)", open(os.path.join(pdir, f)).read())
        assert m and os.path.exists(os.path.join(ROOT, m.group(2))), f
