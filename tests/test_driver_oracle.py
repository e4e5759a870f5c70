"""Pins of the GKBA propagation oracle (oracle/gkba_driver.py).

Each check is independent of the driver's own bookkeeping: a library matrix
exponential for free propagation, the direct collision integral with
exp(-i h (t - t_k)) for frozen h, Hartree and Fock potentials built on a
real-space grid from the definition of the Coulomb integrals (Eq. 3), the
Hubbard and Pariser-Parr-Pople mean fields, the invariants of Eq. 8, and a
self-consistent HF state that must stay stationary without collisions.  Broken
copies of the driver (planted mistakes) must fail one of them.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import gkba_driver as d
from oracle import sb2_oracle as o
from paper_1905_01180_amd import inputs as gen

DT = 0.05


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _system(n, seed, vmax=0.5):
    g = np.random.default_rng(seed)
    h = gen.hermitian_gaussian(n, g)
    v = gen.interaction_lowrank(n, g, vmax=vmax)
    rho0 = gen.density_matrix(n, g)
    return h, v, rho0


# --- free propagation: v = 0 -------------------------------------------------

@pytest.mark.parametrize("hf", [True, False])
def test_free_propagation_closed_form(hf):
    n = 5
    h, v, rho0 = _system(n, 1)
    v = np.zeros_like(v)
    st = d.propagate(v, h, DT, 7, d.new_state(rho0), hf=hf)
    for m in range(8):
        u = scipy.linalg.expm(-1j * h * m * DT)
        assert rel(st["rho"][m], u @ rho0 @ u.conj().T) < 1e-12
    for k in range(7):
        assert rel(st["u"][k], scipy.linalg.expm(-1j * h * (7 - k) * DT)) < 1e-12
    assert np.abs(st["i"]).max() == 0.0


# --- frozen h: the step-by-step history reproduces the direct collision integral

def test_frozen_h_collision_matches_direct_form():
    n = 4
    h, v, rho0 = _system(n, 2)
    st = d.propagate(v, h, DT, 6, d.new_state(rho0), hf=False)
    assert np.abs(st["i"][0]).max() == 0.0
    for m in range(1, 6):                           # I at t_m from rho(t_0..t_{m-1})
        assert rel(st["i"][m], o.collision(v, h, st["rho"][:m], DT)) < 1e-11
    # and the propagators against the plain exponential
    for k in range(6):
        assert rel(st["u"][k], o.propagator(h, (6 - k) * DT)) < 1e-12


# --- Eq. 12 against the definitions of the Hartree and Fock potentials --------

def _grid_system(n, m, seed):
    """Real orthonormal orbitals on m grid points and a real symmetric kernel;
    v_ijkl = sum_{r,r'} phi_i(r) phi_j(r') V(r,r') phi_k(r') phi_l(r) (Eq. 3)."""
    g = np.random.default_rng(seed)
    phi, _ = np.linalg.qr(g.standard_normal((m, n)))          # (r, i)
    x = np.linspace(-3.0, 3.0, m)
    kern = 1.0 / np.sqrt(1.0 + (x[:, None] - x[None, :]) ** 2)
    v = np.einsum("ri,sj,rs,sk,rl->ijkl", phi, phi, kern, phi, phi)
    return phi, kern, v


def test_sigma_hf_equals_grid_hartree_fock():
    n, m = 5, 23
    phi, kern, v = _grid_system(n, m, 3)
    rho = gen.density_matrix(n, np.random.default_rng(4))
    rho_rr = phi @ rho @ phi.T                     # rho(r, r') = sum_lk phi_l(r) rho_lk phi_k(r')
    dens = np.real(np.diagonal(rho_rr))            # n(r) per spin
    v_h = kern @ dens                              # Hartree potential
    hartree = 2.0 * (phi.T * v_h[None, :]) @ phi   # spin factor 2 (closed shell)
    fock = -(phi.T @ (kern * rho_rr) @ phi)        # -V(r,r') rho(r,r')
    assert rel(o.sigma_hf(v, rho), hartree + fock) < 1e-12


def test_sigma_hf_hubbard_and_ppp_mean_fields():
    n = 6
    g = np.random.default_rng(5)
    rho = gen.density_matrix(n, g)
    u = g.uniform(0.5, 2.0, n)
    v_diag = np.zeros((n,) * 4)
    for i in range(n):
        v_diag[i, i, i, i] = u[i]
    # Hubbard: Hartree 2 U n - Fock U n = U n on the diagonal
    assert rel(o.sigma_hf(v_diag, rho), np.diag(u * np.diagonal(rho))) < 1e-14
    vm = g.uniform(0.1, 1.0, (n, n))
    vm = 0.5 * (vm + vm.T)
    v_sym = np.zeros((n,) * 4)
    for i in range(n):
        for j in range(n):
            v_sym[i, j, j, i] = vm[i, j]            # v_ijkl = V_ij delta_il delta_jk
    ppp = 2.0 * np.diag(vm @ np.diagonal(rho)) - vm * rho
    assert rel(o.sigma_hf(v_sym, rho), ppp) < 1e-14


# --- invariants of Eq. 8 -------------------------------------------------------

@pytest.mark.parametrize("hf", [True, False])
def test_hermiticity_and_particle_number(hf):
    n = 4
    h, v, rho0 = _system(n, 6)
    st = d.propagate(v, h, DT, 8, d.new_state(rho0), hf=hf)
    tr0 = np.trace(rho0)
    for r in st["rho"]:
        assert np.abs(r - r.conj().T).max() < 1e-13
        assert abs(np.trace(r) - tr0) < 1e-12
    for u in st["u"]:
        assert np.abs(u @ u.conj().T - np.eye(n)).max() < 1e-12


def _scf_ground_state(h, v, nocc, iters=500):
    rho = np.zeros_like(h)
    rho[np.arange(nocc), np.arange(nocc)] = 1.0
    for _ in range(iters):
        e, p = np.linalg.eigh(h + o.sigma_hf(v, rho))
        new = p[:, :nocc] @ p[:, :nocc].conj().T
        if np.abs(new - rho).max() < 1e-14:
            return new
        rho = 0.5 * rho + 0.5 * new
    return rho


def test_hf_ground_state_is_stationary_without_collisions():
    n = 6
    h, v, _ = _system(n, 7, vmax=0.2)
    rho0 = _scf_ground_state(h, v, 3)
    e, p = np.linalg.eigh(h + o.sigma_hf(v, rho0))
    assert e[3] - e[2] > 1e-3                                   # closed shell
    assert np.abs((h + o.sigma_hf(v, rho0)) @ rho0 - rho0 @ (h + o.sigma_hf(v, rho0))).max() < 1e-12
    st = d.propagate(v, h, DT, 10, d.new_state(rho0), hf=True, collision=False)
    for r in st["rho"]:
        assert np.abs(r - rho0).max() < 1e-11
    # with the bare h in the propagator the same state moves
    st0 = d.propagate(v, h, DT, 3, d.new_state(rho0), hf=False, collision=False)
    assert np.abs(st0["rho"][-1] - rho0).max() > 1e-4


# --- restart from a saved state --------------------------------------------

def test_resume_equals_uninterrupted():
    n = 4
    h, v, rho0 = _system(n, 8)
    full = d.propagate(v, h, DT, 6, d.new_state(rho0))
    part = d.propagate(v, h, DT, 2, d.new_state(rho0))
    part = d.propagate(v, h, DT, 4, part)
    for key in ("rho", "u", "i"):
        assert np.array_equal(full[key], part[key])


# --- planted mistakes ----------------------------------------------------------

def _broken_propagate(v, h, dt, nsteps, rho0, mistake, collision=True):
    rho, u = [rho0], []
    for _ in range(nsteps):
        n = len(rho) - 1
        heff = h + (-o.sigma_hf(v, rho[n]) if mistake == "hf_sign" else o.sigma_hf(v, rho[n]))
        us = o.propagator(heff, dt)
        i_n = d.collision_from_propagators(v, np.stack(u), np.stack(rho[:n]), dt) if n and collision else 0 * h
        hc = i_n if mistake == "no_dagger" else i_n + i_n.conj().T
        rho.append(us @ rho[n] @ us.conj().T - dt * hc)
        u = [(x @ us if mistake == "u_order" else us @ x) for x in u] + [us]
    return np.stack(rho)


def test_planted_mistakes_are_caught():
    n = 4
    h, v, rho0 = _system(n, 9)
    # U history multiplied on the wrong side: breaks the frozen-h direct form
    # (hf=True makes h_HF time dependent so the products do not commute)
    good = d.propagate(v, h, DT, 5, d.new_state(rho0))
    bad = _broken_propagate(v, h, DT, 5, rho0, "u_order")
    assert rel(bad, good["rho"]) > 1e-8
    # collision term without its Hermitian conjugate: rho loses Hermiticity
    bad = _broken_propagate(v, h, DT, 4, rho0, "no_dagger")
    assert max(np.abs(r - r.conj().T).max() for r in bad) > 1e-8
    # HF self-energy with the wrong sign: the SCF state is no longer stationary
    h2, v2, _ = _system(6, 7, vmax=0.2)
    rho_scf = _scf_ground_state(h2, v2, 3)
    assert np.abs(_broken_propagate(v2, h2, DT, 3, rho_scf, "none", collision=False)[-1] - rho_scf).max() < 1e-11
    bad = _broken_propagate(v2, h2, DT, 3, rho_scf, "hf_sign", collision=False)
    assert np.abs(bad[-1] - rho_scf).max() > 1e-6
