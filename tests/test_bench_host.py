"""Host-side logic of bench.py, without a GPU: the algorithmic work and byte counts the roofline is
taken against (their itemised values), the lookup of the recorded HBM traffic (taken only for the
kernel sources and launch configuration the counters were collected on), and the refusal of more
than one GPU."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_peak_is_the_fp32_vector_rate(bench):
    # 256 CUs x 128 FP32 lanes x 2.4 GHz: the published 157.3 TFLOP/s counting an FMA as two
    assert bench.PEAK_VALU_TSLOTS == pytest.approx(157.3 / 2, rel=1e-3)
    assert bench.PEAK_HBM_GBS == 8000.0


@pytest.mark.parametrize("kind,d,r,expected", [
    (0, 1, 1.0, 105.0),      # 1-D LG: 37 noise + 9 model + 13 normalise + 30 resample, adjoint 16
    (0, 1, 0.0, 73.0),       # ... and without resampling
    (3, 1, 0.118, 86.79),    # SV at its resampled fraction (exp in log g and its adjoint)
    (2, 1, 0.82, 121.2),     # growth (a reciprocal in the transition and its slope)
    (1, 16, 0.99, 989.38),   # 16 components: noise, model and adjoint per component
])
def test_algorithmic_slot_counts(bench, kind, d, r, expected):
    assert bench.alg_slots_per_particle_step(0, r, d, kind) == pytest.approx(expected, abs=0.05)


def test_algorithmic_and_design_bytes(bench):
    # a checkpoint every step: the state both ways, the ancestors at resampled steps, the carried
    # log-weight only where the adjoint rebuilds the weights of a step the step before did not
    # resample
    r = 0.25
    assert bench.algorithmic_bytes_per_particle_step(r, 1, 4) == pytest.approx(
        8 * r + 2 * (1 + (1 - r) * r) * 4)
    # every c steps: the state and (unless the step before resampled) the log-weight, each once
    assert bench.algorithmic_bytes_per_particle_step(r, 16, 4) == pytest.approx(
        8 * r + 2 * (1 + 1 - r) * 4 / 16)
    # stored noise adds a write and a read per component
    assert bench.design_bytes_per_particle_step(r, 1, 4, 1) == pytest.approx(
        bench.algorithmic_bytes_per_particle_step(r, 1, 4) + 2 * 4)
    # the segment buffer of the recomputed schedule: state and noise rows, the weight, ancestors
    assert bench.design_bytes_per_particle_step(r, 16, 4, 0) == pytest.approx(
        bench.algorithmic_bytes_per_particle_step(r, 16, 4) + 2 * (2 + r) * 4 + 4 * r)


def test_recorded_traffic_only_for_the_same_kernel_and_configuration(bench, tmp_path,
                                                                    monkeypatch):
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda: "0123456789abcdef")
    rec = dict(kernel_sha="0123456789abcdef", workload="w", tile=3, precision=1, ckpt=1,
               store_noise=0, persistent=1, hbm_bytes_per_launch=123.0)
    with open(tmp_path / "profiles" / "pf_fwd_adj_traffic.json", "w") as f:
        json.dump({"records": [rec]}, f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("w", 3, 1, 1, 0, 1) == 123.0
    for args in [("v", 3, 1, 1, 0, 1), ("w", 4, 1, 1, 0, 1), ("w", 3, 0, 1, 0, 1),
                 ("w", 3, 1, 0, 0, 1), ("w", 3, 1, 1, 1, 1), ("w", 3, 1, 1, 0, 0)]:
        assert bench.recorded_traffic(*args) is None, args
    rec["kernel_sha"] = "0" * 16
    with open(tmp_path / "profiles" / "pf_fwd_adj_traffic.json", "w") as f:
        json.dump({"records": [rec]}, f)
    assert bench.recorded_traffic("w", 3, 1, 1, 0, 1) is None


def test_kernel_hash_ignores_comments_and_layout(bench, tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2407_17296_amd" / "csrc"
    os.makedirs(csrc)
    for name in ("device_common.h", "models.h", "pf_kernel.h"):
        (csrc / name).write_text("int f(int x) { return x + 1; }\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_sources_sha()
    (csrc / "models.h").write_text("// a comment\nint f(int x) {\n  /* and another */ return x + 1;"
                                   "\n}\n")
    assert bench.kernel_sources_sha() == h0
    (csrc / "models.h").write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_sources_sha() != h0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "measures one GPU" in r.stderr
    assert r.stdout.strip() == ""
