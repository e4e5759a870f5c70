"""Autotuner: the tuned launch parameters (and deliberately extreme ones)
change only the schedule, never the result, which stays within the parity
tolerance of the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import sb2_oracle as o
from paper_1905_01180_amd import _lib
from paper_1905_01180_amd import inputs as gen

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-11, "fp32": 2e-6, "fp16x3": 2e-6}


def _case(n, t, sid):
    s = gen.make_system(n, t, config_id=0, system_id=sid)
    want = o.collision(s.v, s.h, s.rho_hist, s.dt)
    dev = torch.device("cuda:0")
    return s, want, [torch.from_numpy(x).to(dev) for x in (s.v, s.h, s.rho_hist)]


def _err(got, want):
    return float(np.abs(got.cpu().numpy() - want).max() / np.abs(want).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x3"])
def test_autotune_then_collision_matches_oracle(prec):
    s, want, (v, h, r) = _case(21, 11, 501)
    print(f"autotune N=21 T=11 {prec}", flush=True)
    cfg = _lib.sb2_autotune(v, h, r, s.dt, prec)
    assert cfg["persist"] in (256, 512, 768, 1024, 1536, 2048, 3072)
    assert cfg["r4pct"] in (50, 100, 150, 200)
    assert cfg["fused"] in ((256, 512, 1024, 2048) if prec == "fp16x3" else (512,))
    got = _lib.sb2_collision(v, h, r, s.dt, prec)
    assert _err(got, want) < TOL[prec]
    _lib.sb2_set_tuning(21, prec)


@pytest.mark.parametrize("persist,r4pct,fused", [(1, 10, 1), (1, 200, 0), (5000, 10, 100000), (5000, 200, 3)])
def test_extreme_tuning_values_keep_results(persist, r4pct, fused):
    s, want, (v, h, r) = _case(19, 6, 502)
    try:
        for prec in ("fp64", "fp32", "fp16x3"):
            print(f"tuning persist={persist} r4pct={r4pct} fused={fused} N=19 T=6 {prec}", flush=True)
            _lib.sb2_set_tuning(19, prec, persist, r4pct, fused)
            got = _lib.sb2_collision(v, h, r, s.dt, prec)
            assert _err(got, want) < TOL[prec], prec
    finally:
        for prec in ("fp64", "fp32", "fp16x3"):
            _lib.sb2_set_tuning(19, prec)
