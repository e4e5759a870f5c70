"""Optional input checks (environment SB2_CHECK=1): a non-Hermitian h or
density matrix and a non-finite interaction are rejected with SB2_ECHECK
before anything else is enqueued; valid inputs give the unchecked result."""
import numpy as np
import pytest

from paper_1905_01180_amd import inputs as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def test_checks_reject_bad_inputs_and_pass_good_ones(monkeypatch):
    from paper_1905_01180_amd import _lib
    s = gen.make_system(12, 6, config_id=230)
    v, h, r = _dev(s.v), _dev(s.h), _dev(s.rho_hist)
    print("case: SB2_CHECK N=12 T=6", flush=True)
    plain = _lib.sb2_collision(v, h, r, s.dt, "fp64")
    monkeypatch.setenv("SB2_CHECK", "1")
    checked = _lib.sb2_collision(v, h, r, s.dt, "fp64")
    assert torch.equal(plain, checked)
    hb = h.clone()
    hb[0, 1] += 1e-3                                   # no longer Hermitian
    with pytest.raises(_lib.Sb2Error) as e:
        _lib.sb2_collision(v, hb, r, s.dt, "fp64")
    assert e.value.status == -7
    rb = r.clone()
    rb[3, 2, 5] += 1e-3j
    with pytest.raises(_lib.Sb2Error) as e:
        _lib.sb2_collision(v, h, rb, s.dt, "fp16x3")
    assert e.value.status == -7
    vb = v.clone()
    vb[1, 2, 3, 4] = float("nan")
    with pytest.raises(_lib.Sb2Error) as e:
        _lib.sb2_sigma(vb, r[:2].clone(), r[2:4].clone(), "fp32")
    assert e.value.status == -7
    with pytest.raises(_lib.Sb2Error) as e:
        _lib.sb2_collision_noalloc(v, hb, r, s.dt, "fp32")
    assert e.value.status == -7
    monkeypatch.setenv("SB2_CHECK", "0")
    _lib.sb2_collision(v, hb, r, s.dt, "fp64")            # unchecked: runs
    torch.cuda.synchronize()
