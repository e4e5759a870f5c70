"""GKBA density-matrix propagation on the device, with checkpoint and resume.

The equation of motion of Sec. II (Eq. 8 with the HF self-energy of Eq. 12,
the GKBA of Eq. 10 and the HF propagators of Eq. 11) is advanced by the HIP
library (sb2_gkba_propagate); this module only owns the device buffers of the
propagation state and writes / reads checkpoints.

State after step n (t_n = n dt):
    rho[k] = rho(t_k),        k = 0..n
    u[k]   = U(t_n, t_k),     k = 0..n-1
    i[m]   = I_ns(t_m),       m = 0..n-1
A checkpoint is these arrays plus (n, dt, precision, included terms) in one
.npz file; resuming continues bit for bit where the saved run stopped.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib

_KEYS = ("rho", "u", "i")


def save_state(path: str, state: dict) -> None:
    """Write a propagation state (numpy arrays and scalars) to an .npz file."""
    check_state(state)
    np.savez(path, n=np.int64(state["n"]), dt=np.float64(state["dt"]), prec=np.str_(state["prec"]),
             hf=np.bool_(state["hf"]), collision=np.bool_(state["collision"]),
             rho=state["rho"], u=state["u"], i=state["i"])


def load_state(path: str) -> dict:
    """Read a state written by save_state (no pickled objects are loaded)."""
    with np.load(path, allow_pickle=False) as z:
        state = {"n": int(z["n"]), "dt": float(z["dt"]), "prec": str(z["prec"]), "hf": bool(z["hf"]),
                 "collision": bool(z["collision"]), "rho": z["rho"].copy(), "u": z["u"].copy(),
                 "i": z["i"].copy()}
    check_state(state)
    return state


def check_state(state: dict) -> None:
    """Shapes of a consistent state: n + 1 densities, n propagators, n collision integrals."""
    n = int(state["n"])
    rho, u, i = (np.asarray(state[k]) for k in _KEYS)
    if n < 0 or rho.ndim != 3 or rho.shape[0] != n + 1 or rho.shape[1] != rho.shape[2]:
        raise ValueError(f"rho must hold n + 1 = {n + 1} square slices, got {rho.shape}")
    nb = rho.shape[1]
    for name, x in (("u", u), ("i", i)):
        if x.shape != (n, nb, nb):
            raise ValueError(f"{name} must have shape {(n, nb, nb)}, got {x.shape}")
    if state["prec"] not in _lib.PRECISIONS:
        raise ValueError(f"unknown precision {state['prec']!r}")
    if not (np.isfinite(state["dt"]) and state["dt"] > 0):
        raise ValueError("dt must be finite and positive")


class GkbaPropagation:
    """Device-resident propagation of one system (v, h fixed; rho evolves).

    capacity: the largest step index the buffers can reach (rho holds
    capacity + 1 slices, u and i capacity slices).
    """

    def __init__(self, v: torch.Tensor, h: torch.Tensor, rho0: torch.Tensor, dt: float, capacity: int,
                 prec: str = "fp64", hf: bool = True, collision: bool = True):
        nb = h.shape[0]
        if capacity < 1:
            raise ValueError("capacity must be >= 1")
        self.v, self.h, self.dt, self.prec = v, h, float(dt), prec
        self.hf, self.collision, self.capacity, self.n = bool(hf), bool(collision), int(capacity), 0
        dev = v.device
        self.rho = torch.zeros((capacity + 1, nb, nb), dtype=torch.complex128, device=dev)
        self.u = torch.zeros((capacity, nb, nb), dtype=torch.complex128, device=dev)
        self.i = torch.zeros((capacity, nb, nb), dtype=torch.complex128, device=dev)
        self.rho[0].copy_(rho0)

    def advance(self, nsteps: int) -> None:
        """Propagate nsteps time steps (one library call, asynchronous on the current stream)."""
        if self.n + nsteps > self.capacity:
            raise ValueError(f"capacity {self.capacity} exceeded by step {self.n + nsteps}")
        _lib.sb2_gkba_propagate(self.v, self.h, self.rho, self.u, self.n, nsteps, self.dt, self.prec,
                                hf=self.hf, collision=self.collision, i_hist=self.i)
        self.n += nsteps

    def state(self) -> dict:
        """Host copy of the current state."""
        n = self.n
        return {"n": n, "dt": self.dt, "prec": self.prec, "hf": self.hf, "collision": self.collision,
                "rho": self.rho[: n + 1].cpu().numpy(), "u": self.u[:n].cpu().numpy(),
                "i": self.i[:n].cpu().numpy()}

    def save(self, path: str) -> None:
        save_state(path, self.state())

    @classmethod
    def resume(cls, path: str, v: torch.Tensor, h: torch.Tensor, capacity: int) -> "GkbaPropagation":
        """Continue a saved propagation with buffers of the given capacity."""
        st = load_state(path)
        n = st["n"]
        if capacity < max(n, 1):
            raise ValueError(f"capacity {capacity} is below the saved step {n}")
        obj = cls(v, h, torch.from_numpy(st["rho"][0]).to(v.device), st["dt"], capacity, st["prec"], st["hf"],
                  st["collision"])
        obj.rho[: n + 1].copy_(torch.from_numpy(st["rho"]))
        obj.u[:n].copy_(torch.from_numpy(st["u"]))
        obj.i[:n].copy_(torch.from_numpy(st["i"]))
        obj.n = n
        return obj
