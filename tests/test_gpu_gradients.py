"""Gradients of L = Im tr[h I_ns] through the hand-written adjoint (C ABI
sb2_collision_backward via the autograd wrapper), checked against
  * torch autograd through the differentiable FP64 CPU oracle (small sizes),
  * central finite differences of the GPU forward (N = 64, T = 256, step 1e-6,
    20 random directions perturbing v, h and rho together).
"""
import numpy as np
import pytest

from paper_1905_01180_amd import inputs as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _grads_gpu(s):
    from paper_1905_01180_amd import autograd as ag
    dev = torch.device("cuda")
    v = torch.from_numpy(s.v).to(dev).requires_grad_(True)
    h = torch.from_numpy(s.h).to(dev).requires_grad_(True)
    r = torch.from_numpy(s.rho_hist).to(dev).requires_grad_(True)
    loss = ag.correlation_observable(v, h, r, s.dt)
    gv, gh, gr = torch.autograd.grad(loss, (v, h, r))
    return float(loss), gv.cpu().numpy(), gh.cpu().numpy(), gr.cpu().numpy()


def _grads_oracle(s):
    from oracle import autograd_oracle as ao
    v = torch.from_numpy(s.v).requires_grad_(True)
    h = torch.from_numpy(s.h).requires_grad_(True)
    r = torch.from_numpy(s.rho_hist).requires_grad_(True)
    loss = ao.correlation_observable(v, h, r, s.dt)
    gv, gh, gr = torch.autograd.grad(loss, (v, h, r))
    return float(loss), gv.numpy(), gh.numpy(), gr.numpy()


def rel(a, b):
    # absolute floor: for N = 1 the collision integral vanishes identically and
    # both gradients are rounding noise (~1e-20)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-8))


@pytest.mark.parametrize("n,t", [(1, 1), (2, 3), (5, 4), (8, 16), (17, 5)])
def test_adjoint_matches_autograd_oracle(n, t):
    s = gen.make_system(n, t, config_id=300, system_id=n)
    print(f"case: gradients vs autograd oracle N={n} T={t}", flush=True)
    lg, gv, gh, gr = _grads_gpu(s)
    lo, ov, oh, orr = _grads_oracle(s)
    assert abs(lg - lo) <= 1e-11 * max(1.0, abs(lo))
    assert rel(gv, ov) < 1e-10, rel(gv, ov)
    assert rel(gh, oh) < 1e-10, rel(gh, oh)
    assert rel(gr, orr) < 1e-10, rel(gr, orr)


def test_adjoint_by_central_differences_c3():
    from paper_1905_01180_amd import _lib
    s = gen.make_config(3)                       # N = 64, T = 256
    print("case: finite differences N=64 T=256", flush=True)
    _, gv, gh, gr = _grads_gpu(s)
    dev = torch.device("cuda")

    def obs(v, h, r):
        i_ns = _lib.sb2_collision(torch.from_numpy(v).to(dev), torch.from_numpy(h).to(dev),
                                  torch.from_numpy(r).to(dev), s.dt, "fp64").cpu().numpy()
        return float(np.trace(h @ i_ns).imag)

    g = np.random.default_rng(33)
    eps = 1e-6
    worst = 0.0
    for d in range(20):
        dv = g.standard_normal(s.v.shape)
        dh = gen.hermitian_gaussian(s.n, g)
        dr = np.stack([gen.hermitian_gaussian(s.n, g) for _ in range(s.t)])
        fd = (obs(s.v + eps * dv, s.h + eps * dh, s.rho_hist + eps * dr)
              - obs(s.v - eps * dv, s.h - eps * dh, s.rho_hist - eps * dr)) / (2 * eps)
        # the observable's explicit h dependence is part of the autograd graph too
        an = (gv * dv).sum() + np.real(np.conj(gh) * dh).sum() + np.real(np.conj(gr) * dr).sum()
        err = abs(fd - an) / max(abs(an), 1e-300)
        worst = max(worst, err)
        print(f"direction {d}: fd={fd:.10e} adjoint={an:.10e} rel={err:.2e}", flush=True)
    assert worst < 1e-6
