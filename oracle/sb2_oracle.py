"""FP64 CPU oracle for the second-Born self-energy and the GKBA collision integral.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU
baseline leg may import or call this module.  It shares no code with the HIP
library (no kernels, headers, helpers, layouts or constants); it reads plain
numpy arrays in the natural index order of the paper and returns them likewise.

Everything is complex128 / float64.  Each function states the passage of
Tuovinen, Covito & Sentef, "Efficient computation of the second-Born
self-energy using tensor-contraction operations" (arXiv:1905.01180) it follows.

Notation (Sec. III): for one pair of times (t, t'),
    G    = G^{<>}(t, t'),   Gbar = G^{><}(t', t),   Sigma = Sigma^{<>}(t, t').
Time grid: t_k = k dt for k = 0..T-1 are the past times, t = T dt is "now".

Readings of the paper taken here (each is listed in the design notes):
  * the quadrature of the time integral in the collision integral (Eq. 9) is the
    left rectangle rule over t_0..t_{T-1} with weight dt (t' = t excluded);
  * the HF propagator of Eq. 11 is evaluated with a frozen one-body matrix h,
    U(t, t') = exp(-i h (t - t')) (the printed lower limit t_0 is read as t');
  * the library-level collision integral I_ns keeps the first two terms of Eq. 9;
    the last two are their Hermitian conjugate, so the paper's I is I_ns + I_ns^dag;
  * the density-matrix step integrates Eq. 8 by exponential Euler (exact
    propagation of the commutator term, explicit Euler for the collision term,
    no predictor-corrector as in Sec. IV).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "propagator", "gkba_pair", "gkba_history", "sigma_naive", "sigma_paper_path",
    "sigma", "exchange_combined", "collision", "collision_paper", "rho_step", "sigma_hf",
    "sigma_diagonal_basis", "sigma_symmetric_basis", "sigma_symmetric_basis_vec",
    "sigma_symmetric_exchange_diag", "collision_with", "vertex_diagonal", "vertex_symmetric",
]


# ---------------------------------------------------------------------------
# Propagators and GKBA two-time functions (Sec. II, Eqs. 8, 10, 11)
# ---------------------------------------------------------------------------

def propagator(h: np.ndarray, tau: float) -> np.ndarray:
    """U = exp(-i h tau) for Hermitian h, through the eigendecomposition of h.

    Eq. 11: G^R(t, t') = -i theta(t - t') U(t, t'); with a time-independent
    (frozen) h the time-ordered exponential is the plain exponential.
    """
    e, p = np.linalg.eigh(h)
    return (p * np.exp(-1j * e * tau)[None, :]) @ p.conj().T


def gkba_pair(u: np.ndarray, rho_k: np.ndarray, rho_t: np.ndarray):
    """GKBA two-time functions between past time t_k and now t (Eq. 10).

    Eq. 10: G^{<>}(t1, t2) = i [G^R(t1, t2) G^{<>}(t2, t2) - G^{<>}(t1, t1) G^A(t1, t2)],
    with G^R(t, t_k) = -i U (Eq. 11), G^A(t_k, t) = G^R(t, t_k)^dag = i U^dag,
    G^R(t_k, t) = G^A(t, t_k) = 0 for t_k < t, and equal-time values
    G^<(s, s) = i rho(s), G^>(s, s) = -i + G^<(s, s) (Sec. II).

    Returns (G^<(t,t_k), G^>(t,t_k), G^<(t_k,t), G^>(t_k,t)).  The now-time
    density rho_t drops out for t_k < t (it multiplies a vanishing propagator)
    and is accepted only to make that visible.
    """
    n = u.shape[0]
    one = np.eye(n)
    gr_t_tk = -1j * u                      # G^R(t, t_k)
    ga_tk_t = gr_t_tk.conj().T             # G^A(t_k, t)
    gr_tk_t = np.zeros_like(u)             # G^R(t_k, t) = 0, t_k < t
    ga_t_tk = np.zeros_like(u)             # G^A(t, t_k) = 0
    gl_kk, gg_kk = 1j * rho_k, -1j * (one - rho_k)
    gl_tt, gg_tt = 1j * rho_t, -1j * (one - rho_t)
    gl_t_tk = 1j * (gr_t_tk @ gl_kk - gl_tt @ ga_t_tk)
    gg_t_tk = 1j * (gr_t_tk @ gg_kk - gg_tt @ ga_t_tk)
    gl_tk_t = 1j * (gr_tk_t @ gl_tt - gl_kk @ ga_tk_t)
    gg_tk_t = 1j * (gr_tk_t @ gg_tt - gg_kk @ ga_tk_t)
    return gl_t_tk, gg_t_tk, gl_tk_t, gg_tk_t


def gkba_history(h: np.ndarray, rho_hist: np.ndarray, dt: float):
    """All GKBA slices for t = T dt against t_k = k dt, k = 0..T-1.

    Returns arrays of shape (T, N, N): U_k, G^<(t,t_k), G^>(t,t_k), G^<(t_k,t), G^>(t_k,t).
    """
    t_len, n, _ = rho_hist.shape
    out = [np.empty((t_len, n, n), np.complex128) for _ in range(5)]
    rho_t = np.zeros((n, n), np.complex128)   # not needed for t_k < t (see gkba_pair)
    for k in range(t_len):
        u = propagator(h, (t_len - k) * dt)
        out[0][k] = u
        for dst, val in zip(out[1:], gkba_pair(u, rho_hist[k], rho_t)):
            dst[k] = val
    return tuple(out)


# ---------------------------------------------------------------------------
# Second-Born self-energy (Sec. III)
# ---------------------------------------------------------------------------

def sigma_naive(v: np.ndarray, g: np.ndarray, gbar: np.ndarray) -> np.ndarray:
    """Eq. 13 written out: the direct (factor 2) minus the exchange term, O(N^8).

    Sigma_ij = 2 sum v_irpn v_mqsj G_nm Gbar_sr G_pq - sum v_irpn v_mqsj G_nq Gbar_sr G_pm,
    summed over m, n, p, q, r, s.  Only for small N.
    """
    direct = np.einsum("irpn,mqsj,nm,sr,pq->ij", v, v, g, gbar, g, optimize=False)
    exchange = np.einsum("irpn,mqsj,nq,sr,pm->ij", v, v, g, gbar, g, optimize=False)
    return 2.0 * direct - exchange


def _c_at_r(c, r):
    # complex @ real through two real BLAS products (keeps the real operand real)
    r = np.ascontiguousarray(r)
    out = np.empty((c.shape[0], r.shape[1]), np.complex128)
    out.real = np.ascontiguousarray(c.real) @ r
    out.imag = np.ascontiguousarray(c.imag) @ r
    return out


def _t1(v, g):
    # T^(1)_nqsj = sum_m v_mqsj G_nm    (Eq. 19)
    n = g.shape[0]
    return _c_at_r(g, v.reshape(n, n ** 3)).reshape(n, n, n, n)


def _t2(v, gbar):
    # T^(2)_ispn = sum_r v_irpn Gbar_sr    (Eq. 19); one product per i
    n = gbar.shape[0]
    out = np.empty((n, n, n, n), np.complex128)
    for i in range(n):
        out[i] = _c_at_r(gbar, v[i].reshape(n, n * n)).reshape(n, n, n)
    return out


def _t3(g, t2):
    # T^(3)_isqn = sum_p G_pq T^(2)_ispn    (Eq. 19); G^T applied to every (i, s) block
    return np.matmul(g.T, t2)


def sigma_paper_path(v: np.ndarray, g: np.ndarray, gbar: np.ndarray) -> np.ndarray:
    """Eq. 19 with the contraction path of Fig. 2: T^(1), T^(2), T^(3), then
    Sigma_ij = sum_nqs (2 T1_nqsj T3_isqn - T1_nqjs T3_isqn).

    The exchange term of Eq. 19 uses v_mqsj = v_qmjs, one of the permutation
    symmetries of Eq. 4, so this form equals Eq. 13 only when v_ijkl = v_jilk.
    """
    n = g.shape[0]
    t1 = _t1(v, g)
    t3 = _t3(g, _t2(v, gbar))
    comb = 2.0 * t1 - t1.transpose(0, 1, 3, 2)                  # (n, q, s, j)
    # sum over (n, q, s): T3[i, s, q, n] * comb[n, q, s, j]
    lhs = t3.transpose(0, 3, 2, 1).reshape(n, n ** 3)           # (i, (n, q, s))
    return lhs @ comb.reshape(n ** 3, n)


def exchange_combined(v: np.ndarray) -> np.ndarray:
    """w_mqsj = 2 v_mqsj - v_qmsj: the two interaction lines of Eq. 13 that meet
    the right-hand vertex, direct and exchange folded together (see sigma)."""
    return 2.0 * v - v.transpose(1, 0, 2, 3)


def sigma(v: np.ndarray, g: np.ndarray, gbar: np.ndarray, w: np.ndarray = None) -> np.ndarray:
    """Eq. 13 regrouped into N^5 contractions without using any symmetry of v.

    Renaming the summation indices m <-> q in the exchange term of Eq. 13 gives
    Sigma_ij = sum v_irpn w_mqsj G_nm G_pq Gbar_sr with w = exchange_combined(v),
    which holds for any v.  It is evaluated on the paper's path (Eq. 19 /
    Fig. 2): T^(1) (here taken on w), T^(2), T^(3), then one sum over (n, q, s).
    w may be passed in to reuse it across many (G, Gbar).
    """
    n = g.shape[0]
    w = exchange_combined(v) if w is None else w
    comb = _t1(w, g)                                             # sum_m w_mqsj G_nm: (n, q, s, j)
    t3 = _t3(g, _t2(v, gbar))                                    # (i, s, q, n)
    lhs = t3.transpose(0, 3, 2, 1).reshape(n, n ** 3)            # (i, (n, q, s))
    return lhs @ comb.reshape(n ** 3, n)


# ---------------------------------------------------------------------------
# Special vertices (Sec. III A, III B): closed forms that pin the general path
# ---------------------------------------------------------------------------

def sigma_diagonal_basis(u_onsite: np.ndarray, g: np.ndarray, gbar: np.ndarray) -> np.ndarray:
    """Eq. 14: for v_ijkl = U_i d_ij d_ik d_il, Sigma_ij = U_i U_j G_ij Gbar_ji G_ij.

    In matrix form (Eq. 15) the on-site factors enter as the outer product
    U U^T; the printed diag(V) o diag(V) is read as that outer product, since
    an entrywise product with diagonal matrices would drop every off-diagonal
    element that Eq. 14 keeps.
    """
    return np.outer(u_onsite, u_onsite) * g * gbar.T * g


def sigma_symmetric_basis(vmat: np.ndarray, g: np.ndarray, gbar: np.ndarray) -> np.ndarray:
    """Eq. 16 for v_ijkl = V_ij d_il d_jk: bubble by the one-liner of Eq. 17,
    exchange by explicit loops over k, l (the off-diagonal part has no
    matrix one-liner, Sec. III B)."""
    n = g.shape[0]
    bubble = 2.0 * g * (vmat @ (vmat @ (gbar.T * g)).T).T
    exch = np.zeros((n, n), np.complex128)
    for i in range(n):
        for j in range(n):
            acc = 0.0j
            for k in range(n):
                for l in range(n):
                    acc += vmat[i, k] * vmat[j, l] * g[i, l] * gbar[l, k] * g[k, j]
            exch[i, j] = -acc
    return bubble + exch


def sigma_symmetric_basis_vec(vmat: np.ndarray, g: np.ndarray, gbar: np.ndarray) -> np.ndarray:
    """Eq. 16 for v_ijkl = V_ij d_il d_jk with both sums as array operations:
    the bubble by Eq. 17, the exchange -sum_kl V_ik V_jl G_il Gbar_lk G_kj as
    one einsum over (k, l) for every (i, j).  Same result as
    sigma_symmetric_basis, O(N^4) without Python loops."""
    bubble = 2.0 * g * (vmat @ (vmat @ (gbar.T * g)).T).T
    exch = -np.einsum("ik,jl,il,lk,kj->ij", vmat, vmat, g, gbar, g, optimize=True)
    return bubble + exch


def sigma_symmetric_exchange_diag(vmat: np.ndarray, g: np.ndarray, gbar: np.ndarray) -> np.ndarray:
    """Eq. 18: diagonal of the exchange term, -diag{(V o G) x [Gbar x (V^T o G)]}."""
    return -np.diagonal((vmat * g) @ (gbar @ (vmat.T * g)))


# ---------------------------------------------------------------------------
# Collision integral and the density-matrix step (Sec. II, Eqs. 8, 9, 12)
# ---------------------------------------------------------------------------

def collision(v: np.ndarray, h: np.ndarray, rho_hist: np.ndarray, dt: float,
              ks=None, return_sigma: bool = False):
    """I_ns(t) = dt sum_k [Sigma^>(t,t_k) G^<(t_k,t) - Sigma^<(t,t_k) G^>(t_k,t)].

    The first two terms of Eq. 9 on the left-rectangle grid t_k = k dt,
    k = 0..T-1, t = T dt; Sigma^< = Sigma(G^<(t,t_k), G^>(t_k,t)) and
    Sigma^> = Sigma(G^>(t,t_k), G^<(t_k,t)) (the naming rule of Sec. III).
    The k-sum runs in k order in float64.

    ks: optional subset of past-time indices (the sum then covers only those).
    return_sigma: also return {k: (Sigma^<_k, Sigma^>_k, term_k)}.
    """
    t_len, n, _ = rho_hist.shape
    ks = range(t_len) if ks is None else ks
    acc = np.zeros((n, n), np.complex128)
    sig = {}
    zero = np.zeros((n, n), np.complex128)
    w = exchange_combined(v)
    for k in ks:
        u = propagator(h, (t_len - k) * dt)
        gl, gg, gl_bar, gg_bar = gkba_pair(u, rho_hist[k], zero)
        s_less = sigma(v, gl, gg_bar, w)
        s_great = sigma(v, gg, gl_bar, w)
        term = s_great @ gl_bar - s_less @ gg_bar
        acc += term
        if return_sigma:
            sig[k] = (s_less, s_great, term * dt)
    acc *= dt
    return (acc, sig) if return_sigma else acc


def collision_with(sigma_fn, h: np.ndarray, rho_hist: np.ndarray, dt: float, return_sigma: bool = False):
    """The collision integral of `collision` with the self-energy of a special
    vertex, sigma_fn(G, Gbar) (Sec. III A, III B): same GKBA functions, same
    naming rule, same k-ordered float64 sum."""
    t_len, n, _ = rho_hist.shape
    acc = np.zeros((n, n), np.complex128)
    zero = np.zeros((n, n), np.complex128)
    sig = {}
    for k in range(t_len):
        u = propagator(h, (t_len - k) * dt)
        gl, gg, gl_bar, gg_bar = gkba_pair(u, rho_hist[k], zero)
        s_less = sigma_fn(gl, gg_bar)
        s_great = sigma_fn(gg, gl_bar)
        acc += s_great @ gl_bar - s_less @ gg_bar
        if return_sigma:
            sig[k] = (s_less, s_great)
    acc *= dt
    return (acc, sig) if return_sigma else acc


def vertex_diagonal(u_onsite: np.ndarray) -> np.ndarray:
    """The diagonal-basis vertex as a full tensor, v_ijkl = U_i d_ij d_ik d_il (Sec. III A)."""
    n = u_onsite.shape[0]
    v = np.zeros((n,) * 4)
    idx = np.arange(n)
    v[idx, idx, idx, idx] = u_onsite
    return v


def vertex_symmetric(vmat: np.ndarray) -> np.ndarray:
    """The symmetric-basis vertex as a full tensor, v_ijkl = V_ij d_il d_jk (Sec. III B)."""
    n = vmat.shape[0]
    v = np.zeros((n,) * 4)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    v[i, j, j, i] = vmat
    return v


def collision_paper(v: np.ndarray, h: np.ndarray, rho_hist: np.ndarray, dt: float) -> np.ndarray:
    """All four terms of Eq. 9, the self-energies at (t_k, t) computed by the
    same 2B formula with the time arguments swapped (not by a symmetry)."""
    t_len, n, _ = rho_hist.shape
    acc = np.zeros((n, n), np.complex128)
    zero = np.zeros((n, n), np.complex128)
    w = exchange_combined(v)
    for k in range(t_len):
        u = propagator(h, (t_len - k) * dt)
        gl, gg, gl_bar, gg_bar = gkba_pair(u, rho_hist[k], zero)
        s_less_t_tk = sigma(v, gl, gg_bar, w)     # Sigma^<(t, t_k)
        s_great_t_tk = sigma(v, gg, gl_bar, w)    # Sigma^>(t, t_k)
        s_less_tk_t = sigma(v, gl_bar, gg, w)     # Sigma^<(t_k, t): G = G^<(t_k,t), Gbar = G^>(t,t_k)
        s_great_tk_t = sigma(v, gg_bar, gl, w)    # Sigma^>(t_k, t)
        acc += (s_great_t_tk @ gl_bar - s_less_t_tk @ gg_bar
                + gl @ s_great_tk_t - gg @ s_less_tk_t)
    return dt * acc


def rho_step(h: np.ndarray, rho: np.ndarray, i_ns: np.ndarray, dt: float) -> np.ndarray:
    """One step of Eq. 8 for rho = -i G^<(t,t).

    With G^<(t,t) = i rho, Eq. 8 reads d rho/dt = -i [h, rho] - I, where
    I = I_ns + I_ns^dag is the full collision integral of Eq. 9.  Exponential
    Euler: rho(t+dt) = U rho U^dag - dt I with U = exp(-i h dt).
    """
    u = propagator(h, dt)
    return u @ rho @ u.conj().T - dt * (i_ns + i_ns.conj().T)


def sigma_hf(v: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """HF self-energy (Eq. 12): (Sigma_HF)_ij = sum_kl (2 v_iklj - v_ikjl) rho_lk."""
    return 2.0 * np.einsum("iklj,lk->ij", v, rho) - np.einsum("ikjl,lk->ij", v, rho)
