"""Pins of the propagation oracle with correlated (quasiparticle) GKBA
propagators (oracle/gkba_driver.propagate(..., sigma_qp=...)).

What fixes the result without the driver's own bookkeeping:
  * a real uniform shift c of the quasiparticle energies multiplies G(t, t_k)
    by exp(-i c (t - t_k)) and the reversed-time functions by the conjugate
    phase; every collision term holds two of each, so the density, the
    collision integral and the HF part are unchanged;
  * a uniform damping gamma multiplies each of the four propagators of a
    collision term (three in the self-energy, one in the closing reversed-time
    function) by exp(-gamma (t - t_k) / 2): term k is weighted by
    exp(-2 gamma (t - t_k)) against the same term built from the HF
    propagators, which the test rebuilds with a library exponential;
  * the reversed-time functions stay minus the adjoints of the forward ones for
    any propagator, so each term conserves the particle number and the density
    keeps its trace (the density step is the unitary HF step).
Two broken drivers (planted mistakes) must fail them."""
import numpy as np
import scipy.linalg

from oracle import gkba_driver as d
from oracle import sb2_oracle as o
from paper_1905_01180_amd import inputs as gen

DT = 0.05


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _system(n, seed, vmax=0.5):
    g = np.random.default_rng(seed)
    return gen.hermitian_gaussian(n, g), gen.interaction_lowrank(n, g, vmax=vmax), gen.density_matrix(n, g)


def _damping(n, seed, scale=0.6):
    g = np.random.default_rng(seed)
    x = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    gam = x @ x.conj().T
    return scale * gam / np.abs(gam).max()               # Hermitian positive semidefinite


def test_zero_correction_is_the_hf_propagation():
    h, v, rho0 = _system(5, 1)
    plain = d.propagate(v, h, DT, 6, d.new_state(rho0))
    qp = d.propagate(v, h, DT, 6, d.new_state(rho0), sigma_qp=np.zeros((5, 5), complex))
    for key in ("rho", "i", "u"):
        assert rel(qp[key], plain[key]) < 1e-12


def test_real_uniform_shift_leaves_the_dynamics_unchanged():
    n, c, steps = 5, 0.7, 7
    h, v, rho0 = _system(n, 2)
    plain = d.propagate(v, h, DT, steps, d.new_state(rho0))
    qp = d.propagate(v, h, DT, steps, d.new_state(rho0), sigma_qp=c * np.eye(n))
    assert rel(qp["rho"], plain["rho"]) < 1e-12
    assert rel(qp["i"][1:], plain["i"][1:]) < 1e-11
    for k in range(steps):                               # the propagators carry the phase
        assert rel(qp["u"][k], np.exp(-1j * c * (steps - k) * DT) * plain["u"][k]) < 1e-12


def _hf_history(v, h, rho, m):
    """HF propagators U(t_m, t_k), k < m, rebuilt from a density history."""
    steps = [scipy.linalg.expm(-1j * DT * (h + o.sigma_hf(v, rho[j]))) for j in range(m)]
    out = []
    for k in range(m):
        u = np.eye(h.shape[0], dtype=complex)
        for j in range(k, m):
            u = steps[j] @ u
        out.append(u)
    return out


def _weighted_collision(v, h, rho, m, gamma):
    u = _hf_history(v, h, rho, m)
    acc = 0
    for k in range(m):
        term = d.collision_from_propagators(v, u[k][None], rho[k:k + 1], DT)
        acc = acc + np.exp(-2.0 * gamma * (m - k) * DT) * term
    return acc


def test_uniform_damping_weights_each_past_time():
    n, gamma, steps = 4, 0.8, 6
    h, v, rho0 = _system(n, 3)
    qp = d.propagate(v, h, DT, steps, d.new_state(rho0), sigma_qp=-0.5j * gamma * np.eye(n))
    for m in range(1, steps):
        assert rel(qp["i"][m], _weighted_collision(v, h, qp["rho"], m, gamma)) < 1e-11


def test_damped_propagation_keeps_trace_and_hermiticity():
    n, steps = 5, 8
    h, v, rho0 = _system(n, 4)
    sq = -0.5j * _damping(n, 5) + 0.1 * gen.hermitian_gaussian(n, np.random.default_rng(6))
    qp = d.propagate(v, h, DT, steps, d.new_state(rho0), sigma_qp=sq)
    for r in qp["rho"]:
        assert abs(np.trace(r) - np.trace(rho0)) < 1e-12
        assert np.abs(r - r.conj().T).max() < 1e-13
    assert rel(qp["rho"][-1], d.propagate(v, h, DT, steps, d.new_state(rho0))["rho"][-1]) > 1e-6


def _broken(v, h, rho0, steps, sq, mistake):
    """The driver with one planted mistake; returns (rho history, I history)."""
    rho, u, ih = [rho0], [], []
    for _ in range(steps):
        n = len(rho) - 1
        heff = h + o.sigma_hf(v, rho[n])
        us = o.propagator(heff, DT)
        uq = scipy.linalg.expm(-1j * DT * (heff + sq))
        i_n = d.collision_from_propagators(v, np.stack(u), np.stack(rho[:n]), DT) if n else 0 * h
        ur = uq if mistake == "damped_density" else us
        rho.append(ur @ rho[n] @ ur.conj().T - DT * (i_n + i_n.conj().T))
        ih.append(i_n)
        u = [(us if mistake == "newest_only" else uq) @ x for x in u] + [uq]
    return np.stack(rho), np.stack(ih)


def test_planted_mistakes_are_caught():
    n, gamma, steps = 4, 0.8, 5
    h, v, rho0 = _system(n, 3)
    sq = -0.5j * gamma * np.eye(n)
    # density advanced with the damped step: the trace decays
    rho_b, _ = _broken(v, h, rho0, steps, sq, "damped_density")
    assert abs(np.trace(rho_b[-1]) - np.trace(rho0)) > 1e-3
    # older history entries advanced with the HF step: past time k keeps only
    # one damped step, so the weights of the damping pin are missed
    rho_b, i_b = _broken(v, h, rho0, steps, sq, "newest_only")
    assert rel(i_b[1], _weighted_collision(v, h, rho_b, 1, gamma)) < 1e-11   # one past time: no difference
    assert max(rel(i_b[m], _weighted_collision(v, h, rho_b, m, gamma)) for m in range(2, steps)) > 1e-3
