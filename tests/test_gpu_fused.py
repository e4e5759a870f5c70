"""The fused second/third contraction (split float16, N <= 112) against the
FP64 oracle and against the two-launch path on the same inputs, at basis sizes
on both sides of every 16- and 32-wide tile edge the kernel has (one to seven
waves, one to four 32-row slabs, ragged tails), plus a case that uses the
two-launch path because N is above the fused kernel's limit."""
import numpy as np
import pytest

from oracle import sb2_oracle as o
from paper_1905_01180_amd import inputs as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TOL = 2e-6


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("n,b", [(1, 2), (15, 2), (16, 3), (31, 2), (32, 1), (33, 2), (48, 1), (63, 1), (70, 1),
                                 (81, 1), (96, 2), (97, 1), (100, 1), (100, 3), (101, 2), (112, 1), (112, 2),
                                 (113, 1)])
def test_fused_matches_oracle_and_two_launch_path(n, b):
    from paper_1905_01180_amd import _lib
    g = np.random.default_rng(3000 + n)
    v = gen.interaction_generic(n, g)
    gl = g.standard_normal((b, n, n)) + 1j * g.standard_normal((b, n, n))
    gg = g.standard_normal((b, n, n)) + 1j * g.standard_normal((b, n, n))
    print(f"case: fused sigma N={n} B={b}", flush=True)
    try:
        _lib.sb2_set_tuning(n, "fp16x3", fused=512)
        fl, fg = (x.cpu().numpy() for x in _lib.sb2_sigma(dev(v), dev(gl), dev(gg), "fp16x3"))
        _lib.sb2_set_tuning(n, "fp16x3", fused=0)
        sl, sg = (x.cpu().numpy() for x in _lib.sb2_sigma(dev(v), dev(gl), dev(gg), "fp16x3"))
    finally:
        _lib.sb2_set_tuning(n, "fp16x3")
    for k in range(b):
        want_l = o.sigma(v, gl[k], -gg[k].conj().T)
        want_g = o.sigma(v, gg[k], -gl[k].conj().T)
        assert rel(fl[k], want_l) < TOL, (k, rel(fl[k], want_l))
        assert rel(fg[k], want_g) < TOL, (k, rel(fg[k], want_g))
        assert rel(sl[k], want_l) < TOL
        assert rel(sg[k], want_g) < TOL
        assert rel(fl[k], sl[k]) < TOL


def test_fused_zero_input_gives_zero():
    from paper_1905_01180_amd import _lib
    n = 40
    v = np.zeros((n, n, n, n))
    g = np.random.default_rng(7)
    gl = g.standard_normal((2, n, n)) + 1j * g.standard_normal((2, n, n))
    sl, sg = _lib.sb2_sigma(dev(v), dev(gl), dev(gl.copy()), "fp16x3")
    assert float(sl.abs().max()) == 0.0 and float(sg.abs().max()) == 0.0
