"""FP64 CPU oracle for the GKBA time propagation of the density matrix.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU
baseline leg may import or call this module.  It shares no code with the HIP
library; it builds on the plain formulas of sb2_oracle.

The propagation follows Sec. II of Tuovinen, Covito & Sentef
(arXiv:1905.01180):
  * Eq. 8: i d/dt G^<(t,t) = [h + Sigma_HF, G^<(t,t)] + I(t) with
    G^<(t,t) = i rho(t), i.e. d rho/dt = -i [h_HF, rho] - I, I = I_ns + I_ns^dag;
  * Eq. 12: the time-local HF self-energy from the density matrix;
  * Eq. 11: the HF propagators as the time-ordered exponential of h + Sigma_HF;
  * Eq. 10: the GKBA two-time functions from those propagators and the
    equal-time functions of the past times;
  * Sec. IV: a time-stepping scheme without predictor-corrector.

Time-dependent coupling (adiabatic switching, Sec. II: a correlated state is
prepared by starting uncorrelated and slowly switching the interaction on):
with H(t) = h + lambda(t) V, the HF self-energy at t_n carries lambda(t_n)
and the second-Born self-energy Sigma(t_n, t_k), whose two interaction lines
sit at t_n and at t_k, carries lambda(t_n) lambda(t_k).

Readings (also listed in the design notes):
  * time grid t_n = n dt; at step n the collision integral sums the past times
    t_0..t_{n-1} with weight dt (left rectangle, t' = t excluded); at n = 0 it
    is zero;
  * h_HF is sampled at the start of each step, h_HF(t_n) = h + Sigma_HF(rho_n),
    and the time-ordered exponential over [t_k, t_n] is the product of the step
    exponentials U_step(n-1) ... U_step(k), U_step(m) = exp(-i h_HF(t_m) dt);
  * the density step is exponential Euler with the same U_step(n):
    rho_{n+1} = U_step(n) rho_n U_step(n)^dag - dt (I_n + I_n^dag).
"""
from __future__ import annotations

import numpy as np

from .sb2_oracle import exchange_combined, gkba_pair, propagator, sigma, sigma_hf

__all__ = ["collision_from_propagators", "propagate", "new_state"]


def collision_from_propagators(v: np.ndarray, u_hist: np.ndarray, rho_hist: np.ndarray, dt: float,
                               lam=None, lam_now: float = 1.0) -> np.ndarray:
    """I_ns(t) = dt sum_k [Sigma^>(t,t_k) G^<(t_k,t) - Sigma^<(t,t_k) G^>(t_k,t)].

    The first two terms of Eq. 9 with the GKBA functions of Eq. 10 built from
    given propagators u_hist[k] = U(t, t_k) (Eq. 11) and rho_hist[k] = rho(t_k);
    Sigma^< = Sigma(G^<(t,t_k), G^>(t_k,t)), Sigma^> = Sigma(G^>(t,t_k), G^<(t_k,t))
    as in Sec. III.  The k-sum runs in k order.  With a time-dependent coupling
    lambda (lam[k] = lambda(t_k), lam_now = lambda(t)) each self-energy is
    multiplied by lam_now lam[k].
    """
    t_len, n, _ = u_hist.shape
    acc = np.zeros((n, n), np.complex128)
    if t_len == 0:
        return acc
    zero = np.zeros((n, n), np.complex128)
    w = exchange_combined(v)
    for k in range(t_len):
        gl, gg, gl_bar, gg_bar = gkba_pair(u_hist[k], rho_hist[k], zero)
        s_less = sigma(v, gl, gg_bar, w)
        s_great = sigma(v, gg, gl_bar, w)
        c = 1.0 if lam is None else lam_now * lam[k]
        acc += c * (s_great @ gl_bar - s_less @ gg_bar)
    return dt * acc


def new_state(rho0: np.ndarray) -> dict:
    """Propagation state at t_0: rho history [rho_0], no propagators, no I yet."""
    n = rho0.shape[0]
    return {
        "rho": np.asarray(rho0, np.complex128).reshape(1, n, n).copy(),
        "u": np.zeros((0, n, n), np.complex128),
        "i": np.zeros((0, n, n), np.complex128),
    }


def propagate(v: np.ndarray, h: np.ndarray, dt: float, nsteps: int, state: dict,
              hf: bool = True, collision: bool = True, switch=None) -> dict:
    """Advance the GKBA state by nsteps time steps (returns a new state).

    state["rho"][k] = rho(t_k) for k = 0..n, state["u"][k] = U(t_n, t_k) for
    k = 0..n-1, state["i"][m] = I_ns(t_m) for m = 0..n-1.
    hf: include Sigma_HF (Eq. 12) in the propagator and the commutator.
    collision: include the 2B collision integral (Eq. 9).
    switch: optional coupling lambda(t_m) for every step index m the run
    reaches (the interaction is lambda(t) V; see the module notes).
    """
    rho = list(state["rho"])
    u = [x.copy() for x in state["u"]]
    ihist = list(state["i"])
    for _ in range(nsteps):
        n = len(rho) - 1
        rho_n = rho[n]
        lam_n = 1.0 if switch is None else float(switch[n])
        h_eff = h + lam_n * sigma_hf(v, rho_n) if hf else h.copy()
        u_step = propagator(h_eff, dt)
        if collision and n > 0:
            i_n = collision_from_propagators(v, np.stack(u), np.stack(rho[:n]), dt,
                                             None if switch is None else switch, lam_n)
        else:
            i_n = np.zeros_like(rho_n)
        rho.append(u_step @ rho_n @ u_step.conj().T - dt * (i_n + i_n.conj().T))
        ihist.append(i_n)
        u = [u_step @ x for x in u] + [u_step]
    nn = rho[0].shape[0]
    return {
        "rho": np.stack(rho),
        "u": np.stack(u) if u else np.zeros((0, nn, nn), np.complex128),
        "i": np.stack(ihist) if ihist else np.zeros((0, nn, nn), np.complex128),
    }
