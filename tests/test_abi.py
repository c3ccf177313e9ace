"""The C-ABI library loads and exports every entry point include/smc2.h declares; host-side
validation answers with status codes (no GPU needed for these)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2407_17296_amd import smc2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smc2.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smc2_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(smc2.LIB_PATH):
        from paper_2407_17296_amd import build
        build.build()
    return smc2.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    # and the binding wraps each of them under the same name
    wrapped = {s[0] for s in smc2.SIGNATURES}
    assert set(names) == wrapped


def test_version_string(lib):
    assert "gfx950" in smc2.smc2_version()


def test_scratch_bytes_follow_the_layout(lib):
    m = smc2.Model(smc2.LG1D, 1, 3)
    o = smc2.pf_opts(precision=smc2.FP64, ckpt_interval=16)
    b = smc2.smc2_ctx_scratch_bytes(m, o, 1, 1024, 1024, 250)
    # ancestors int32 [1024][250][1024] dominate; checkpoints [16 segs][2][1024] FP64 per item
    assert b >= 1024 * 250 * 1024 * 4 + 1024 * 16 * 2 * 1024 * 8
    o32 = smc2.pf_opts(precision=smc2.MIXED, ckpt_interval=16)
    assert smc2.smc2_ctx_scratch_bytes(m, o32, 1, 1024, 1024, 250) < b


@pytest.mark.parametrize("bad", [
    dict(kind=smc2.LG1D, d=1, D=4),
    dict(kind=smc2.LG_DIAG, d=8, D=10),
    dict(kind=9, d=1, D=3),
])
def test_bad_models_are_rejected(lib, bad):
    m = smc2.Model(bad["kind"], bad["d"], bad["D"])
    with pytest.raises(smc2.SMC2Error) as e:
        smc2.smc2_ctx_scratch_bytes(m, smc2.pf_opts(), 1, 1, 64, 10)
    assert e.value.status == smc2.SMC2_E_INVALID_ARG


def test_bad_options_and_sizes_are_rejected(lib):
    m = smc2.Model(smc2.GROWTH, 1, 2)
    with pytest.raises(smc2.SMC2Error) as e:
        smc2.smc2_ctx_scratch_bytes(m, smc2.pf_opts(precision=7), 1, 1, 64, 10)
    assert e.value.status == smc2.SMC2_E_UNSUPPORTED
    with pytest.raises(smc2.SMC2Error):
        smc2.smc2_ctx_scratch_bytes(m, smc2.pf_opts(ess_frac=-1.0), 1, 1, 64, 10)
    with pytest.raises(smc2.SMC2Error):
        smc2.smc2_ctx_scratch_bytes(m, smc2.pf_opts(), 0, 1, 64, 10)
    with pytest.raises(smc2.SMC2Error) as e:
        smc2.smc2_ctx_scratch_bytes(m, smc2.pf_opts(), 1, 1, 8192, 10)
    assert e.value.status == smc2.SMC2_E_UNSUPPORTED
    bad_prior = smc2.Model(smc2.GROWTH, 1, 2, prior_sd=[1.0, 0.0])
    with pytest.raises(smc2.SMC2Error):
        smc2.smc2_ctx_scratch_bytes(bad_prior, smc2.pf_opts(), 1, 1, 64, 10)


def test_filter_regions_beyond_32_bit_offsets_are_refused(lib):
    # a filter's stored noise is (T+1) x d x M_pow2 values: at d=16, M=2048 in FP64 that is
    # 256 KiB per step, so 16383 steps reach 4 GiB and no longer fit 32-bit byte offsets
    m = smc2.Model(smc2.LG_DIAG, 16, 18)
    o = smc2.pf_opts(precision=smc2.FP64, ckpt_interval=0, store_noise=1)
    assert smc2.smc2_ctx_scratch_bytes(m, o, 1, 1, 2048, 16382) > 0
    with pytest.raises(smc2.SMC2Error) as e:
        smc2.smc2_ctx_scratch_bytes(m, o, 1, 1, 2048, 16383)
    assert e.value.status == smc2.SMC2_E_UNSUPPORTED
    assert "4 GiB" in str(e.value)
    # regenerating the noise stores none: the checkpoints (sqrt(T) rows) stay far below
    o_regen = smc2.pf_opts(precision=smc2.FP64, ckpt_interval=0, store_noise=0)
    assert smc2.smc2_ctx_scratch_bytes(m, o_regen, 1, 1, 2048, 16383) > 0
    # a checkpoint at every step: (T+1) rows of (d+1) x M_pow2 values reach 4 GiB first
    o_every = smc2.pf_opts(precision=smc2.FP64, ckpt_interval=1, store_noise=0)
    assert smc2.smc2_ctx_scratch_bytes(m, o_every, 1, 1, 2048, 15419) > 0
    with pytest.raises(smc2.SMC2Error):
        smc2.smc2_ctx_scratch_bytes(m, o_every, 1, 1, 2048, 15420)


def test_tile_table(lib):
    for t in range(1, 17):
        mp, w, p = smc2.smc2_tile_info(t, 1)
        assert mp == 64 * w * p
    mp, w, p = smc2.smc2_tile_info(17, 16)
    assert (mp, w, p) == (2048, 16, 2)
    with pytest.raises(smc2.SMC2Error):
        smc2.smc2_tile_info(99, 1)


def test_no_device_is_an_error_not_a_crash(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(smc2.SMC2Error) as e:
        smc2.smc2_ctx_create(0)
    assert e.value.status in (smc2.SMC2_E_INVALID_ARG, smc2.SMC2_E_DEVICE)


def test_product_path_does_not_touch_the_oracle():
    """The package never imports or loads the oracle, and fails loudly without its library."""
    pkg = os.path.join(ROOT, "paper_2407_17296_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "pyoracle" not in src and "liboracle" not in src and "orc_" not in src, f
    code = open(os.path.join(pkg, "smc2.py")).read()
    assert "raise RuntimeError" in code and "not built" in code


def test_sir_model_and_priors_are_validated(lib):
    """The SIR model takes d_x = 2, d_y = 1, D = 2; its constants and uniform priors are
    checked before anything is reserved."""
    o = smc2.pf_opts()
    ok = smc2.Model(smc2.SIR, 2, 2, [0.0, 0.0], [1.0, 1.0],
                    prior_kind=[smc2.PRIOR_UNIFORM] * 2)
    assert smc2.smc2_ctx_scratch_bytes(ok, o, 1, 64, 250, 35) > 0
    with_c = smc2.Model(smc2.SIR, 2, 2, [0.0, 0.0], [1.0, 1.0],
                        prior_kind=[smc2.PRIOR_UNIFORM] * 2, constants=[500.0, 5.0, 0.5, 2.0])
    assert smc2.smc2_ctx_scratch_bytes(with_c, o, 1, 64, 250, 35) > 0
    bad = [
        smc2.Model(smc2.SIR, 1, 2),                                          # d_x
        smc2.Model(smc2.SIR, 2, 2, constants=[100.0, 200.0, 0.5, 5.0]),      # I_0 > N_pop
        smc2.Model(smc2.SIR, 2, 2, constants=[100.0, 1.0, -0.5, 5.0]),       # negative variance
        smc2.Model(smc2.SIR, 2, 2, constants=[100.0, 1.0, 0.5, 0.0]),        # s_y = 0
        smc2.Model(smc2.SIR, 2, 2, constants=[np.inf, 1.0, 0.5, 5.0]),       # non-finite
        smc2.Model(smc2.SIR, 2, 2, [0.0, 1.0], [1.0, 1.0],
                   prior_kind=[smc2.PRIOR_UNIFORM] * 2),                      # empty interval
        smc2.Model(smc2.SIR, 2, 2, prior_kind=[0, 7]),                       # unknown kind
    ]
    for m in bad:
        with pytest.raises(smc2.SMC2Error) as e:
            smc2.smc2_ctx_scratch_bytes(m, o, 1, 64, 250, 35)
        assert e.value.status == smc2.SMC2_E_INVALID_ARG
    # two-component states are built up to 2048 particles
    with pytest.raises(smc2.SMC2Error) as e:
        smc2.smc2_ctx_scratch_bytes(ok, o, 1, 1, 4096, 35)
    assert e.value.status == smc2.SMC2_E_UNSUPPORTED


def test_sir_tiles_are_built(lib):
    for t in (1, 2, 3, 4, 6, 7, 10, 11, 14, 17):
        mp, w, p = smc2.smc2_tile_info(t, 2)
        assert mp == 64 * w * p
    with pytest.raises(smc2.SMC2Error):
        smc2.smc2_tile_info(8, 2)  # 16 particles per lane is not built for two components


def test_calls_without_a_reserved_context_are_refused(lib):
    """The outer-step calls take their device from a reserved context and refuse a missing one
    with a status, before touching any device."""
    m = smc2.Model(smc2.LG1D, 1, 3)
    mp = ctypes.byref(m.c)
    assert lib.smc2_langevin_move(None, mp, 1, 4, 0.1, 0, None, None, 1, None, None, None,
                                  None) == smc2.SMC2_E_INVALID_ARG
    assert lib.smc2_prior_init(None, mp, 1, 4, 1, None, None) == smc2.SMC2_E_INVALID_ARG
    assert lib.smc2_reweight_resample(None, mp, 1, 4, 0.1, 0, None, None, None, 1, 1, None, 0,
                                      None, None, None, None, None,
                                      None) == smc2.SMC2_E_INVALID_ARG
    assert b"reserved" in lib.smc2_last_error()
