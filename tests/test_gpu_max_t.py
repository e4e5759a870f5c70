"""The longest history the library accepts (T = SB2_MAX_T = 65536 past
times, t = T dt = 3276.8) at a small basis (N = 4), against the full FP64
oracle: index arithmetic over the longest propagator and density histories,
the chunking of the past times and the float64 sum over all of them.

Bars: the device builds U(t, t_k) by repeated doubling of one step, the oracle
by eigendecomposition, so the propagators differ by about T eps_mach
(7e-12); float64 is held to 1e-10 and split float16 to 2e-6, both relative to
the sum over past times of each term's max-abs size, which bounds any error
that is relative to the terms whether they cancel or accumulate."""
import numpy as np
import pytest

from oracle import sb2_oracle as o
from paper_1905_01180_amd import inputs as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
T_MAX = 65536
_ref = {}


def _case():
    if not _ref:
        s = gen.make_system(4, T_MAX, config_id=7, system_id=1)
        print(f"oracle: N=4 T={T_MAX} (full sum)", flush=True)
        want, sig = o.collision(s.v, s.h, s.rho_hist, s.dt, return_sigma=True)
        scale = sum(np.abs(t).max() for _, _, t in sig.values())
        _ref.update(s=s, want=want, scale=scale)
    return _ref["s"], _ref["want"], _ref["scale"]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp16x3", 2e-6)])
def test_collision_at_max_t(prec, tol):
    from paper_1905_01180_amd import _lib
    s, want, scale = _case()
    dev = torch.device("cuda:0")
    print(f"case: collision N=4 T={T_MAX} {prec}", flush=True)
    got = _lib.sb2_collision(torch.from_numpy(s.v).to(dev), torch.from_numpy(s.h).to(dev),
                             torch.from_numpy(s.rho_hist).to(dev), s.dt, prec).cpu().numpy()
    err = np.abs(got - want).max() / scale
    print(f"max T {prec}: err {err:.2e} of the summed term size (|I| / that {np.abs(want).max() / scale:.2e})",
          flush=True)
    assert err < tol
