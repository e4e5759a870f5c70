"""Differentiable FP64 CPU oracle (torch, complex128) for gradient checks.

TEST INFRASTRUCTURE.  Only the tests may import this module.  It restates the
same passages as sb2_oracle in torch operations so that torch's autograd can
differentiate a scalar observable of the collision integral with respect to
v, h and the density history; it imports nothing from the HIP library.

Gradient convention: torch's, grad = dL/dRe z + i dL/dIm z for complex inputs
(so the directional derivative along d is Re sum conj(grad) * d).
"""
from __future__ import annotations

import torch


def propagator(h: torch.Tensor, tau: float) -> torch.Tensor:
    """U = exp(-i h tau) (Eq. 11 with a frozen h), by torch's matrix exponential."""
    return torch.linalg.matrix_exp(-1j * tau * h)


def sigma(v: torch.Tensor, g: torch.Tensor, gbar: torch.Tensor) -> torch.Tensor:
    """Eq. 13 with the exchange term's dummy indices renamed (m <-> q):
    Sigma_ij = sum v_irpn (2 v_mqsj - v_qmsj) G_nm G_pq Gbar_sr."""
    w = 2.0 * v - v.permute(1, 0, 2, 3)
    vc, wc = v.to(g.dtype), w.to(g.dtype)
    a = torch.einsum("nm,mqsj->nqsj", g, wc)
    b = torch.einsum("pq,nqsj->npsj", g, a)
    c = torch.einsum("sr,npsj->nprj", gbar, b)
    return torch.einsum("irpn,nprj->ij", vc, c)


def collision(v: torch.Tensor, h: torch.Tensor, rho_hist: torch.Tensor, dt: float) -> torch.Tensor:
    """I_ns = dt sum_k [Sigma^>_k G^<(t_k,t) - Sigma^<_k G^>(t_k,t)] (Eq. 9, first two
    terms, left-rectangle grid t_k = k dt, t = T dt), GKBA slices from Eq. 10."""
    t_len, n, _ = rho_hist.shape
    eye = torch.eye(n, dtype=h.dtype)
    acc = torch.zeros((n, n), dtype=h.dtype)
    for k in range(t_len):
        u = propagator(h, (t_len - k) * dt)
        rho = rho_hist[k]
        gl = 1j * (u @ rho)                              # G^<(t, t_k) = G^R G^<(t_k,t_k) i
        gg = -1j * (u @ (eye - rho))                     # G^>(t, t_k)
        gl_bar = 1j * (rho @ u.conj().T)                 # G^<(t_k, t) = -G^<(t_k,t_k) G^A i
        gg_bar = -1j * ((eye - rho) @ u.conj().T)        # G^>(t_k, t)
        acc = acc + sigma(v, gg, gl_bar) @ gl_bar - sigma(v, gl, gg_bar) @ gg_bar
    return dt * acc


def correlation_observable(v, h, rho_hist, dt) -> torch.Tensor:
    """The scalar L = Im tr[h I_ns] used for the gradient checks."""
    i_ns = collision(v, h, rho_hist, dt)
    return torch.diagonal(h @ i_ns).sum().imag
