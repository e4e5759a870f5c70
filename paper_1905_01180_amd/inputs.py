"""Seeded synthetic inputs for the second-Born / GKBA collision-integral path.

This module only draws random numbers and builds input tensors (h, v, rho
history) with the structure the method expects.  It holds none of the method's
arithmetic: no propagator, no GKBA two-time function, no self-energy, no
collision integral.  Both the FP64 oracle's tests and the HIP path's tests and
benchmark take their inputs from here, so the two see identical bits.

Structure of the inputs (the paper's model, Sec. II):
  * h      -- one-body Hermitian matrix h_ij (Eq. 1-2).  Here (X + X^dag)/2 with
              X_ij = a + ib, a, b ~ N(0, 1): E|h_ij|^2 = 1 off the diagonal and a
              real N(0, 1) diagonal.
  * v      -- real two-body tensor v_ijkl (Eq. 3).  For a real basis it has the
              8-fold permutation symmetry of Eq. 4 (pairs {i, l} and {j, k}).
              "lowrank" (the workloads' default, the construction the workloads
              name): X_ijkl = sum_g A_ig A_jg B_kg B_lg, v = (X + X_klij)/2,
              scaled to max|v| = 0.5.  It has {ijkl, jilk, klij, lkji} but also
              i <-> j alone and k <-> l alone, which are NOT symmetries of Eq. 4;
              with them the exchange term of Eq. 13 is exactly -1/2 of the direct
              term, so checks that must separate the two use one of the others:
              "generic" averages an i.i.d. Gaussian tensor over {ijkl, jilk,
              klij, lkji} (no low-rank structure, no i <-> j symmetry), and
              "orbitals" builds Coulomb-like integrals of real orthonormal
              functions on a grid (exactly the 8-fold symmetry of Eq. 4).
  * rho    -- one-particle density matrix, Hermitian with eigenvalues in [0, 1]
              and trace N/2 (rho = -i G^<(t,t), Sec. II).  Eigenvalues come in
              pairs (u, 1-u) with u ~ U[0,1] (plus 0.5 when N is odd), rotated by
              a Haar unitary.
  * history -- rho_k for k = 0..T-1.  "smooth": rho_k = R_k rho_0 R_k^dag with
              R_k a seeded unitary path exp(-i H k dt) for an independent random
              Hermitian H (so the spectrum and trace stay fixed and the history
              is as smooth as a real propagation); "iid": an independent rho per k.

Seeds: numpy Generator(PCG64(SeedSequence([1905, 1180, config, system, stream]))).
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

SEED_PREFIX = (1905, 1180)
DT_DEFAULT = 0.05

# stream ids: one independent random stream per generated object
_S_H, _S_V, _S_RHO0, _S_HIST, _S_DIR = 0, 1, 2, 3, 4


def rng(config_id: int, system_id: int, stream_id: int) -> np.random.Generator:
    """Independent, reproducible random stream for one generated object."""
    ss = np.random.SeedSequence([*SEED_PREFIX, int(config_id), int(system_id), int(stream_id)])
    return np.random.Generator(np.random.PCG64(ss))


def hermitian_gaussian(n: int, g: np.random.Generator) -> np.ndarray:
    x = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    return 0.5 * (x + x.conj().T)


def interaction_lowrank(n: int, g: np.random.Generator, vmax: float = 0.5) -> np.ndarray:
    """Dense real v_ijkl with v_ijkl = v_jilk = v_klij = v_lkji, max|v| = vmax.

    Also symmetric under i <-> j alone and k <-> l alone (not symmetries of
    real-orbital integrals): then 2 v_mqsj - v_qmsj = v_mqsj, and the exchange
    term of Eq. 13 is exactly -1/2 of the direct term.  Index-order checks of
    the exchange term need interaction_generic or interaction_real_orbitals."""
    a = g.standard_normal((n, n))
    b = g.standard_normal((n, n))
    aa = (a[:, None, :] * a[None, :, :]).reshape(n * n, n)      # (ij, g)
    bb = (b[:, None, :] * b[None, :, :]).reshape(n * n, n)      # (kl, g)
    x = (aa @ bb.T).reshape(n, n, n, n)                          # X_ijkl
    v = 0.5 * (x + x.transpose(2, 3, 0, 1))                      # + X_klij
    v *= vmax / np.abs(v).max()
    return np.ascontiguousarray(v)


def interaction_generic(n: int, g: np.random.Generator, vmax: float = 0.5) -> np.ndarray:
    """Full-rank real v averaged over the sub-group {ijkl, jilk, klij, lkji}."""
    x = g.standard_normal((n, n, n, n))
    v = 0.25 * (x + x.transpose(1, 0, 3, 2) + x.transpose(2, 3, 0, 1) + x.transpose(3, 2, 1, 0))
    v *= vmax / np.abs(v).max()
    return np.ascontiguousarray(v)


def interaction_real_orbitals(n: int, g: np.random.Generator, m: int = 0, vmax: float = 0.5) -> np.ndarray:
    """Real v_ijkl = sum_{r,r'} phi_i(r) phi_j(r') K(r,r') phi_k(r') phi_l(r) from n
    orthonormal real functions on m grid points and K(r,r') = 1/sqrt(1+(x-x')^2):
    the full 8-point symmetry of real orbitals; max|v| = vmax."""
    m = m or 2 * n + 8
    phi, _ = np.linalg.qr(g.standard_normal((m, n)))
    x = np.linspace(-3.0, 3.0, m)
    kern = 1.0 / np.sqrt(1.0 + (x[:, None] - x[None, :]) ** 2)
    f = (phi[:, :, None] * phi[:, None, :]).reshape(m, n * n)       # f[r, (a,b)] = phi_a(r) phi_b(r)
    x_ab_cd = f.T @ kern @ f                                         # [(i,l), (j,k)]
    v = x_ab_cd.reshape(n, n, n, n).transpose(0, 2, 3, 1)            # (i,l,j,k) -> (i,j,k,l)
    v *= vmax / np.abs(v).max()
    return np.ascontiguousarray(v)


def haar_unitary(n: int, g: np.random.Generator) -> np.ndarray:
    z = (g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def density_matrix(n: int, g: np.random.Generator) -> np.ndarray:
    """Hermitian rho with eigenvalues uniform in [0,1] and trace exactly n/2."""
    u = g.uniform(0.0, 1.0, size=n // 2)
    lam = np.concatenate([u, 1.0 - u, [0.5] if n % 2 else []])
    q = haar_unitary(n, g)
    rho = (q * lam[None, :]) @ q.conj().T
    return 0.5 * (rho + rho.conj().T)


def unitary_path(hr: np.ndarray, taus: np.ndarray) -> np.ndarray:
    """exp(-i hr tau) for every tau (a smooth path of unitaries, for synthetic states)."""
    return _unitary_path(hr, np.asarray(taus, dtype=np.float64))


def _unitary_path(hr: np.ndarray, taus: np.ndarray) -> np.ndarray:
    e, p = np.linalg.eigh(hr)
    ph = np.exp(-1j * e[None, :] * taus[:, None])                # (K, n)
    return np.einsum("ia,ka,ja->kij", p, ph, p.conj())


def rho_history(n: int, t: int, dt: float, g: np.random.Generator, kind: str = "smooth") -> np.ndarray:
    if kind == "iid":
        return np.stack([density_matrix(n, g) for _ in range(t)])
    if kind != "smooth":
        raise ValueError(f"unknown history kind {kind!r}")
    rho0 = density_matrix(n, g)
    hr = hermitian_gaussian(n, g)
    r = _unitary_path(hr, dt * np.arange(t, dtype=np.float64))
    hist = r @ rho0[None] @ r.conj().transpose(0, 2, 1)
    return np.ascontiguousarray(0.5 * (hist + hist.conj().transpose(0, 2, 1)))


def chain_hopping(n: int, hop: float = -1.0) -> np.ndarray:
    """Open chain of n sites with nearest-neighbour hopping `hop` (h_ij = hop for |i - j| = 1)."""
    h = np.zeros((n, n), np.complex128)
    idx = np.arange(n - 1)
    h[idx, idx + 1] = hop
    h[idx + 1, idx] = hop
    return h


def hubbard_onsite(n: int, u: float = 1.0) -> np.ndarray:
    """On-site interaction U_i = u of the diagonal (Hubbard) basis."""
    return np.full(n, float(u))


def ohno_matrix(n: int, u: float = 1.0) -> np.ndarray:
    """Long-range interaction of the Ohno model, V_ij = u / sqrt(1 + |i - j|^2)."""
    idx = np.arange(n)
    return u / np.sqrt(1.0 + (idx[:, None] - idx[None, :]) ** 2.0)


def left_half_density(n: int) -> np.ndarray:
    """Density matrix with the n // 2 leftmost sites filled and the rest empty:
    the state that a strong confinement potential on the left half gives with
    n // 2 particles per spin."""
    return np.diag(np.concatenate([np.ones(n // 2), np.zeros(n - n // 2)])).astype(np.complex128)


@dataclasses.dataclass
class System:
    """One synthetic GKBA system: frozen h, dense real v, rho history, dt."""
    n: int
    t: int
    dt: float
    h: np.ndarray          # (n, n) complex128, Hermitian
    v: np.ndarray          # (n, n, n, n) float64
    rho_hist: np.ndarray   # (t, n, n) complex128, rho_hist[k] = rho(k dt)

    @property
    def flops(self) -> float:
        """Algorithmic real flops of one collision-integral evaluation (48 T N^5)."""
        return 48.0 * self.t * float(self.n) ** 5


def make_system(n: int, t: int, config_id: int = 0, system_id: int = 0, dt: float = DT_DEFAULT,
                v_kind: str = "lowrank", hist_kind: str = "smooth") -> System:
    h = hermitian_gaussian(n, rng(config_id, system_id, _S_H))
    gv = rng(config_id, system_id, _S_V)
    if v_kind == "lowrank":
        v = interaction_lowrank(n, gv)
    elif v_kind == "generic":
        v = interaction_generic(n, gv)
    elif v_kind == "orbitals":
        v = interaction_real_orbitals(n, gv)
    else:
        raise ValueError(f"unknown interaction kind {v_kind!r}")
    hist = rho_history(n, t, dt, rng(config_id, system_id, _S_HIST), hist_kind)
    return System(n=n, t=t, dt=dt, h=h, v=v, rho_hist=hist)


# The five workloads: (config id, N, T).  Config 4 is a batch of 32 systems.
CONFIGS = {
    0: dict(n=10, t=20),      # plain method, oracle in full
    1: dict(n=50, t=500),     # FP64 baseline
    2: dict(n=100, t=1000),   # precision workload (headline)
    3: dict(n=64, t=256),     # differentiation
}


def make_config(config_id: int, **kw) -> System:
    return make_system(config_id=config_id, **CONFIGS[config_id], **kw)


def batch_shapes(nsys: int = 32, config_id: int = 4, n_range=(24, 96), t_range=(64, 512)) -> List[tuple]:
    """(N_b, T_b) for a batched workload: N ~ U{n_range}, T ~ U{t_range}
    (defaults: the 32-system workload, N 24..96, T 64..512)."""
    g = rng(config_id, 0, _S_DIR)
    ns = g.integers(n_range[0], n_range[1] + 1, size=nsys)
    ts = g.integers(t_range[0], t_range[1] + 1, size=nsys)
    return [(int(a), int(b)) for a, b in zip(ns, ts)]


def make_batch(nsys: int = 32, config_id: int = 4, shapes=None, n_range=(24, 96), t_range=(64, 512)) -> List[System]:
    shapes = shapes if shapes is not None else batch_shapes(nsys, config_id, n_range, t_range)
    return [make_system(n, t, config_id=config_id, system_id=i + 1) for i, (n, t) in enumerate(shapes)]


def hermitian_directions(n: int, count: int, seed: int = 0) -> np.ndarray:
    g = rng(3, seed, _S_DIR)
    return np.stack([hermitian_gaussian(n, g) for _ in range(count)])
