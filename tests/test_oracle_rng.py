"""Pins of the oracle's counter-based random numbers (Philox4x32-10 + Box-Muller).

The paper needs random numbers that are fixed per filter (common random numbers, Sec. II-A),
drawn in advance (App. A, eq. reparam_epsilon) and, for resampling, uniform on (0, 1] and
independent per particle and step (App. B).  The counter contract realises that; these tests pin
the oracle's implementation to an independent one and to distributional facts.
"""
import os
import subprocess

import numpy as np
import pytest
from scipy import stats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REF_SRC = os.path.join(ROOT, "tests", "philox_rocrand_ref.cpp")
REF_BIN = os.path.join(ROOT, "tests", "_build", "philox_rocrand_ref")


def _rocrand_ref(rows):
    """Philox words from rocRAND's host-callable engine (an implementation independent of ours)."""
    if not os.path.exists(REF_BIN) or os.path.getmtime(REF_BIN) < os.path.getmtime(REF_SRC):
        os.makedirs(os.path.dirname(REF_BIN), exist_ok=True)
        subprocess.check_call(["hipcc", "-O1", "-x", "hip", "--offload-arch=gfx950",
                               "-I/opt/rocm/include", "-o", REF_BIN, REF_SRC],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
    out = subprocess.run([REF_BIN], input=inp, capture_output=True, text=True, check=True).stdout
    return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64)


def test_philox_matches_rocrand(oracle):
    rng = np.random.default_rng(1)
    rows = []
    for _ in range(200):
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        c[1] = c[1] % (2**30)  # rocRAND's offset argument is 4*counter and must not wrap
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        rows.append(list(c) + list(k))
    rows.append([0, 0, 0, 0, 0, 0])
    ref = _rocrand_ref(rows)
    for r, want in zip(rows, ref):
        got = oracle.philox(r[:4], r[4:])
        assert np.array_equal(got.astype(np.uint64), want), (r, got, want)


def test_box_muller_word_mapping(oracle):
    """Normal n uses Box-Muller pair p = n//2 from block p//2, words 2(p%2), 2(p%2)+1."""
    seed = 0x0123456789ABCDEF
    c0, c2, c3 = 7, 11, oracle.c3(3, oracle.STEP_NORMAL)
    rows = [[c0, b, c2, c3, seed & 0xFFFFFFFF, seed >> 32] for b in range(4)]
    words = _rocrand_ref(rows)
    for n in range(16):
        p = n // 2
        w = words[p // 2]
        u1 = (float(w[2 * (p % 2)]) + 1.0) * 2.0**-32
        u2 = float(w[2 * (p % 2) + 1]) * 2.0**-32
        r = np.sqrt(-2.0 * np.log(u1))
        want = r * (np.sin(2 * np.pi * u2) if n % 2 else np.cos(2 * np.pi * u2))
        assert oracle.lib().orc_normal(seed, c0, c2, c3, n) == pytest.approx(want, rel=1e-14, abs=1e-14)
    for m in range(16):
        w = words[m // 4]
        want = (float(w[m % 4]) + 1.0) * 2.0**-32
        assert oracle.lib().orc_uniform(seed, c0, c2, c3, m) == want


def test_normals_are_standard_normal(oracle):
    z = oracle.normals(17296, 3, 5, oracle.c3(1, oracle.STEP_NORMAL), 0, 200_000)
    n = len(z)
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # pairs of one Box-Muller draw and neighbouring slots are uncorrelated
    z2 = oracle.normals(17296, 4, 5, oracle.c3(1, oracle.STEP_NORMAL), 0, 200_000)
    assert abs(np.corrcoef(z, z2)[0, 1]) < 5 / np.sqrt(n)
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 5 / np.sqrt(n / 2)


def test_uniforms_on_half_open_interval(oracle):
    u = oracle.uniforms(99, 0xFFFFFFFF, 0, oracle.c3(2, oracle.RESAMPLE_UNIFORM), 0, 200_000)
    assert u.min() > 0.0 and u.max() <= 1.0
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / len(u))
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_streams_distinct_by_every_counter_field(oracle):
    base = dict(seed=5, c0=1, c2=2, c3=oracle.c3(1, oracle.STEP_NORMAL))
    ref = oracle.normals(base["seed"], base["c0"], base["c2"], base["c3"], 0, 64)
    for field, val in (("seed", 6), ("c0", 2), ("c2", 3), ("c3", oracle.c3(2, oracle.STEP_NORMAL)),
                       ("c3", oracle.c3(1, oracle.INIT_NORMAL))):
        kw = dict(base)
        kw[field] = val
        other = oracle.normals(kw["seed"], kw["c0"], kw["c2"], kw["c3"], 0, 64)
        assert not np.allclose(ref, other)
