"""The device's counter-based random numbers equal the oracle's: Philox words bit-exact, FP64
normals to rounding, uniforms exact (the common-random-numbers contract, Sec. II-A)."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def test_device_philox_equals_oracle(oracle):
    import torch
    from paper_2407_17296_amd import smc2
    rng = np.random.default_rng(0)
    R = 4096
    ctr = rng.integers(0, 2**32, size=(R, 4), dtype=np.uint64)
    ctr[:8] = [[0, 0, 0, 0], [2**32 - 1] * 4, [5, 0, 7, 0x102], [0, 1, 2, 3],
               [0xFFFFFFFF, 9, 3, 0x203], [1, 2, 3, 4], [7, 0, 0, 0x301], [0, 0, 1, 0]]
    n = rng.integers(0, 4096, size=R, dtype=np.uint64)
    ctr[:, 1] = n // 4  # the probe draws normal / uniform n from the block of its counter
    seed = 0x0123456789ABCDEF
    say("  philox probe R=%d" % R)
    dev = torch.device("cuda:0")
    tc = torch.tensor(ctr.astype(np.uint32).view(np.int32), device=dev)
    tn = torch.tensor(n.astype(np.uint32).view(np.int32), device=dev)
    out, nz, un, nz32, un32 = smc2.smc2_philox_probe(tc, tn, seed)
    torch.cuda.synchronize()
    out = out.cpu().numpy().view(np.uint32)
    nz, un, nz32, un32 = (a.cpu().numpy() for a in (nz, un, nz32, un32))
    key = [seed & 0xFFFFFFFF, seed >> 32]
    lib = oracle.lib()
    for r in range(R):
        want = oracle.philox(ctr[r], key)
        assert np.array_equal(out[r], want), r
    c0, c2, c3 = ctr[:, 0], ctr[:, 2], ctr[:, 3]
    on = np.array([lib.orc_normal(seed, int(c0[r]), int(c2[r]), int(c3[r]), int(n[r])) for r in range(R)])
    ou = np.array([lib.orc_uniform(seed, int(c0[r]), int(c2[r]), int(c3[r]), int(n[r])) for r in range(R)])
    assert np.array_equal(un, ou)
    assert np.max(np.abs(nz - on) / np.maximum(1.0, np.abs(on))) < 1e-14
    assert np.max(np.abs(nz32 - on)) < 2e-5 * np.max(np.abs(on))
    assert np.max(np.abs(un32 - ou)) < 1e-7
    say("  max |normal64 - oracle| %.2e, max |normal32 - oracle| %.2e" % (
        np.max(np.abs(nz - on)), np.max(np.abs(nz32 - on))))
