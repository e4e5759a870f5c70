"""Pin of the density-matrix equation of motion against exact many-body dynamics.

The sign and weight of the collision term in the density step (Eq. 8 with the
collision integral of Eq. 9, the GKBA of Eq. 10 and the 2B self-energy of
Eq. 13) are fixed here by physics, not by restating the paper's algebra:

* the second-Born self-energy holds every self-energy diagram of second order
  in the interaction (the first-order HF diagrams with the dressed G, the
  second-order direct and exchange diagrams), so its Kadanoff-Baym dynamics is
  exact through O(v^2);
* the collision integral is already O(v^2), so it needs the two-time functions
  only at zeroth order, where the GKBA reconstruction from the density is exact
  (free propagation of a non-interacting state); from an uncorrelated
  (Slater-determinant) initial state there is no initial-correlation term.

Hence the O(v^2) part of rho(t) from the GKBA propagation must converge, as
dt -> 0, to the O(v^2) part of the exact rho(t) of the spin-1/2 many-body
Hamiltonian H = sum h_ij c+_is c_js + 1/2 sum v_ijkl c+_is c+_jt c_kt c_ls
(Eqs. 1-3), obtained here by exact diagonalisation in Fock space.  The
collision term contributes about a quarter of that O(v^2) part on these
systems, so a flipped or dropped collision term, a wrong factor of the direct
or exchange term, or a wrong GKBA sign fails; the O(v) part pins the HF
self-energy of Eq. 12 the same way.

Orders in v come from central differences in the coupling lambda (v -> lambda
v) with one Richardson step; the time-step error of the propagation (first
order in dt) is removed by one Richardson step over dt and dt/2, and the
remainder must shrink like dt^2.
"""
import numpy as np
import pytest

from oracle import gkba_driver as d
from oracle import sb2_oracle as o
from paper_1905_01180_amd import inputs as gen

TIMES = (0.5, 1.0)
DTS = (0.05, 0.025, 0.0125)
EPS = 0.02


# --- exact dynamics in Fock space -------------------------------------------

def _annihilators(m):
    """Jordan-Wigner matrices of c_p on the 2^m-dimensional Fock space; bit p of
    a basis index is the occupation of mode p."""
    dim = 1 << m
    ops = []
    for p in range(m):
        c = np.zeros((dim, dim))
        for s in range(dim):
            if s >> p & 1:
                c[s ^ (1 << p), s] = (-1) ** bin(s & ((1 << p) - 1)).count("1")
        ops.append(c)
    return ops


def exact_density(h, v, orbitals, times):
    """rho_ij(t) = <c+_j,up c_i,up> for the state that starts as the Slater
    determinant with the columns of `orbitals` doubly occupied (mode 2 i + s
    is orbital i with spin s)."""
    n = h.shape[0]
    c = _annihilators(2 * n)
    cd = [x.T for x in c]
    dim = 1 << (2 * n)
    ham = np.zeros((dim, dim), complex)
    for i in range(n):
        for j in range(n):
            for s in range(2):
                ham += h[i, j] * cd[2 * i + s] @ c[2 * j + s]
    for i, j, k, l in np.ndindex(n, n, n, n):
        if v[i, j, k, l] != 0.0:
            for s in range(2):
                for t in range(2):
                    ham += 0.5 * v[i, j, k, l] * cd[2 * i + s] @ cd[2 * j + t] @ c[2 * k + t] @ c[2 * l + s]
    assert np.abs(ham - ham.conj().T).max() < 1e-12
    psi = np.zeros(dim, complex)
    psi[0] = 1.0
    for a in range(orbitals.shape[1]):
        for s in range(2):
            psi = sum(orbitals[i, a] * cd[2 * i + s] for i in range(n)) @ psi
    psi /= np.linalg.norm(psi)
    e, p = np.linalg.eigh(ham)
    coef = p.conj().T @ psi
    out = []
    for t in times:
        pt = p @ (np.exp(-1j * e * t) * coef)
        out.append([[pt.conj() @ (cd[2 * j] @ c[2 * i] @ pt) for j in range(n)] for i in range(n)])
    return np.array(out)


# --- orders in the coupling and in dt -----------------------------------------

def order1(fn):
    r = {x: fn(x) for x in (EPS, -EPS, 2 * EPS, -2 * EPS)}
    d1 = (r[EPS] - r[-EPS]) / (2 * EPS)
    d2 = (r[2 * EPS] - r[-2 * EPS]) / (4 * EPS)
    return (4 * d1 - d2) / 3


def order2(fn):
    r = {x: fn(x) for x in (0.0, EPS, -EPS, 2 * EPS, -2 * EPS)}
    d1 = (r[EPS] + r[-EPS] - 2 * r[0.0]) / EPS ** 2
    d2 = (r[2 * EPS] + r[-2 * EPS] - 2 * r[0.0]) / (2 * EPS) ** 2
    return (4 * d1 - d2) / 6


def _idx(dt):
    return [int(round(t / dt)) for t in TIMES]


def driver_rho(v, h, rho0, dt, hf=True, collision=True):
    idx = _idx(dt)
    return d.propagate(v, h, dt, idx[-1], d.new_state(rho0), hf=hf, collision=collision)["rho"][idx]


def driver_flipped(v, h, rho0, dt):
    """The propagation oracle with the collision term's sign flipped (planted mistake)."""
    idx = _idx(dt)
    rho, u = [rho0], []
    for n in range(idx[-1]):
        us = o.propagator(h + o.sigma_hf(v, rho[n]), dt)
        i_n = d.collision_from_propagators(v, np.stack(u), np.stack(rho[:n]), dt) if n else 0 * h
        rho.append(us @ rho[n] @ us.conj().T + dt * (i_n + i_n.conj().T))
        u = [us @ x for x in u] + [us]
    return np.stack(rho)[idx]


def frozen_h_rho(v, h, rho0, dt, sign=1.0):
    """Collision-only propagation from the single-evaluation functions:
    rho_{n+1} = rho_step(h, rho_n, I_n) with I_n = collision(v, h, rho_0..rho_{n-1})
    (bare h, no HF self-energy); sign=-1 plants a flipped collision term."""
    idx = _idx(dt)
    rho = [rho0]
    for n in range(idx[-1]):
        i_n = o.collision(v, h, np.stack(rho[:n]), dt) if n else 0 * h
        rho.append(o.rho_step(h, rho[n], sign * i_n, dt))
    return np.stack(rho)[idx]


def richardson(fn):
    """First-order-in-dt extrapolations over (DTS[0], DTS[1]) and (DTS[1], DTS[2])."""
    vals = [fn(dt) for dt in DTS]
    return 2 * vals[1] - vals[0], 2 * vals[2] - vals[1]


def _case(n, nocc, seed):
    g = np.random.default_rng(seed)
    h = gen.hermitian_gaussian(n, g)
    v = gen.interaction_real_orbitals(n, g)
    z = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    orb = np.linalg.qr(z)[0][:, :nocc]
    return h, v, orb, orb @ orb.conj().T


CASES = [(3, 1, 5), (3, 2, 6)]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"n{c[0]}occ{c[1]}")
def case(request):
    n, nocc, seed = request.param
    h, v, orb, rho0 = _case(n, nocc, seed)
    ex1 = order1(lambda lam: exact_density(h, lam * v, orb, TIMES))
    ex2 = order2(lambda lam: exact_density(h, lam * v, orb, TIMES))
    mf2 = richardson(lambda dt: order2(lambda lam: driver_rho(lam * v, h, rho0, dt, collision=False)))[1]
    return dict(h=h, v=v, rho0=rho0, ex1=ex1, ex2=ex2, coll2=ex2 - mf2)


def _err(a, b):
    return float(np.abs(a - b).max())


def test_first_order_density_is_exact_hf(case):
    h, v, rho0 = case["h"], case["v"], case["rho0"]
    r_coarse, r_fine = richardson(lambda dt: order1(lambda lam: driver_rho(lam * v, h, rho0, dt)))
    scale = np.abs(case["ex1"]).max()
    e_c, e_f = _err(r_coarse, case["ex1"]), _err(r_fine, case["ex1"])
    print(f"O(v): |rho1| {scale:.3e}, extrapolated errors {e_c:.3e} -> {e_f:.3e}")
    assert e_f < 0.02 * scale and e_f < 0.4 * e_c


def test_second_order_density_is_exact(case):
    h, v, rho0 = case["h"], case["v"], case["rho0"]
    r_coarse, r_fine = richardson(lambda dt: order2(lambda lam: driver_rho(lam * v, h, rho0, dt)))
    coll = np.abs(case["coll2"]).max()
    e_c, e_f = _err(r_coarse, case["ex2"]), _err(r_fine, case["ex2"])
    print(f"O(v^2): |rho2| {np.abs(case['ex2']).max():.3e}, collision part {coll:.3e}, "
          f"extrapolated errors {e_c:.3e} -> {e_f:.3e}")
    assert coll > 0.1 * np.abs(case["ex2"]).max()       # the collision term matters here
    assert e_f < 0.15 * coll and e_f < 0.4 * e_c
    # planted mistake: the collision term with the opposite sign
    bad = richardson(lambda dt: order2(lambda lam: driver_flipped(lam * v, h, rho0, dt)))[1]
    assert _err(bad, case["ex2"]) > 1.0 * coll


def test_collision_and_rho_step_give_the_exact_correlation_part(case):
    # with the bare h the O(v^2) density is the collision term's part alone (the
    # HF terms start at O(v), their cross terms with the collision term at O(v^3))
    h, v, rho0 = case["h"], case["v"], case["rho0"]
    want = case["coll2"]
    got = richardson(lambda dt: order2(lambda lam: frozen_h_rho(lam * v, h, rho0, dt)))[1]
    scale = np.abs(want).max()
    print(f"correlation part {scale:.3e}, error {_err(got, want):.3e}")
    assert _err(got, want) < 0.2 * scale
    bad = richardson(lambda dt: order2(lambda lam: frozen_h_rho(lam * v, h, rho0, dt, sign=-1.0)))[1]
    assert _err(bad, want) > 1.5 * scale


# --- time-dependent coupling (adiabatic switching) ----------------------------
#
# With H(t) = h + lambda(t) V the second-Born self-energy Sigma(t, t') carries
# lambda(t) lambda(t') (one interaction line at each time) and the HF
# self-energy lambda(t): the switched propagation must again agree with exact
# dynamics through O(v^2).  Placing lambda(t)^2 or lambda(t')^2 on Sigma
# instead (planted below) must not.

def ramp(t):
    """A coupling that varies on the time scale of the collision integral's
    memory (a slow switch-on would hide where lambda sits): on from zero,
    then oscillating."""
    return np.sin(0.5 * np.pi * min(t, 0.3) / 0.3) ** 2 * (1.0 + 0.6 * np.sin(2.0 * np.pi * t / 0.6))


def exact_density_switched(h, v, orbitals, times, dt_exact=0.0025):
    """As exact_density for H(t) = h + ramp(t) V, stepped with the midpoint
    exponential of H (second order in dt_exact)."""
    n = h.shape[0]
    c = _annihilators(2 * n)
    cd = [x.T for x in c]
    dim = 1 << (2 * n)
    h1 = np.zeros((dim, dim), complex)
    for i in range(n):
        for j in range(n):
            for s in range(2):
                h1 += h[i, j] * cd[2 * i + s] @ c[2 * j + s]
    h2 = np.zeros((dim, dim))
    for i, j, k, l in np.ndindex(n, n, n, n):
        if v[i, j, k, l] != 0.0:
            for s in range(2):
                for t in range(2):
                    h2 += 0.5 * v[i, j, k, l] * cd[2 * i + s] @ cd[2 * j + t] @ c[2 * k + t] @ c[2 * l + s]
    psi = np.zeros(dim, complex)
    psi[0] = 1.0
    for a in range(orbitals.shape[1]):
        for s in range(2):
            psi = sum(orbitals[i, a] * cd[2 * i + s] for i in range(n)) @ psi
    psi /= np.linalg.norm(psi)
    out, t = [], 0.0
    for target in times:
        steps = int(round((target - t) / dt_exact))
        for _ in range(steps):
            e, p = np.linalg.eigh(h1 + ramp(t + 0.5 * dt_exact) * h2)
            psi = p @ (np.exp(-1j * e * dt_exact) * (p.conj().T @ psi))
            t += dt_exact
        out.append([[psi.conj() @ (cd[2 * j] @ c[2 * i] @ psi) for j in range(n)] for i in range(n)])
    return np.array(out)


def switched_rho(v, h, rho0, dt, weight="product"):
    """Switched propagation; weight='product' is the oracle, the others are
    planted mistakes (lambda(t_n)^2 or lambda(t_k)^2 on Sigma(t_n, t_k))."""
    idx = _idx(dt)
    lam = np.array([ramp(m * dt) for m in range(idx[-1] + 1)])
    if weight == "product":
        return d.propagate(v, h, dt, idx[-1], d.new_state(rho0), switch=lam)["rho"][idx]
    rho, u = [rho0], []
    for n in range(idx[-1]):
        us = o.propagator(h + lam[n] * o.sigma_hf(v, rho[n]), dt)
        if n:
            w = np.full(n, lam[n]) if weight == "now" else lam[:n]
            i_n = d.collision_from_propagators(v, np.stack(u), np.stack(rho[:n]), dt, w,
                                               lam[n] if weight == "now" else 1.0)
            if weight == "past":
                i_n = d.collision_from_propagators(v, np.stack(u), np.stack(rho[:n]), dt, lam[:n] ** 2, 1.0)
        else:
            i_n = 0 * h
        rho.append(us @ rho[n] @ us.conj().T - dt * (i_n + i_n.conj().T))
        u = [us @ x for x in u] + [us]
    return np.stack(rho)[idx]


def richardson2(fn):
    """Two Richardson steps over DTS (removing the dt and dt^2 terms)."""
    vals = [fn(dt) for dt in DTS]
    r1, r2 = 2 * vals[1] - vals[0], 2 * vals[2] - vals[1]
    return (4 * r2 - r1) / 3


def test_switched_coupling_is_exact_through_second_order():
    h, v, orb, rho0 = _case(3, 1, 5)
    ex2 = order2(lambda lam: exact_density_switched(h, lam * v, orb, TIMES))
    err = {w: _err(richardson2(lambda dt: order2(lambda lam: switched_rho(lam * v, h, rho0, dt, w))), ex2)
           for w in ("product", "now", "past")}
    scale = np.abs(ex2).max()
    print(f"switched O(v^2): |rho2| {scale:.3e}, extrapolated error {err['product']:.3e}; "
          f"lambda(t)^2: {err['now']:.3e}, lambda(t')^2: {err['past']:.3e}")
    assert err["product"] < 0.01 * scale
    assert err["now"] > 5 * err["product"] and err["past"] > 5 * err["product"]
