"""The allocation-free collision entry point (static per-device scratch
buffer) against sb2_collision with a caller workspace, through the C ABI: two
calls in a row on the same buffer, the second smaller than the first, at all
three precisions.  The first call does not fit the buffer in one pass, so it
also runs several chunks of past times.  Bars: float64 1e-11, float32 and split
float16 2e-6 (max-abs error over max-abs value; the chunking changes only the
order of float32 accumulation)."""
import numpy as np
import pytest

from paper_1905_01180_amd import inputs as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 2e-6, "fp16x3": 2e-6}


def rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x3"])
def test_noalloc_matches_workspace_entry_point(prec):
    from paper_1905_01180_amd import _lib
    dev = torch.device("cuda:0")
    for n, t, sid in ((24, 40, 1), (10, 9, 2)):
        s = gen.make_system(n, t, config_id=220, system_id=sid)
        v, h, r = (torch.from_numpy(x).to(dev) for x in (s.v, s.h, s.rho_hist))
        print(f"case: noalloc N={n} T={t} {prec}", flush=True)
        want, wsig = _lib.sb2_collision(v, h, r, s.dt, prec, return_sigma=True)
        got, gsig = _lib.sb2_collision_noalloc(v, h, r, s.dt, prec, return_sigma=True)
        torch.cuda.synchronize()
        e_i, e_s = rel(got, want), rel(gsig, wsig)
        print(f"noalloc N={n} T={t} {prec}: rel diff I {e_i:.2e}, Sigma {e_s:.2e}", flush=True)
        assert e_i < TOL[prec] and e_s < TOL[prec]
