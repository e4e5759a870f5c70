"""ctypes binding of libsb2.so (argument marshalling only).

Every computation runs in the HIP library; this module checks tensor shapes,
dtypes and devices, hands device pointers and the current HIP stream to the
C ABI and keeps one reusable device workspace per (device, stream).  It fails loudly if
the library is not built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsb2.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sb2.h")

PRECISIONS = {"fp64": 0, "fp32": 1, "fp16x3": 2, "bf16x6": 3}   # bf16x6: recognised, not built
OPS = {"sigma": 0, "collision": 1, "collision_backward": 2, "rho_step": 3, "autotune": 4, "propagate": 5,
       "collision_diagonal": 6, "collision_symmetric": 7, "propagate_diagonal": 8, "propagate_symmetric": 9,
       "propagate_linear": 10}
VERTICES = {"diagonal": 1, "symmetric": 2}
PROP_HF, PROP_COLLISION = 1, 2
STATUS = {0: "SB2_OK", -1: "SB2_EINVAL", -2: "SB2_ESHAPE", -3: "SB2_EWORKSPACE", -4: "SB2_EHIP",
          -5: "SB2_EUNSUPPORTED", -6: "SB2_ESCRATCH",
          -7: "SB2_ECHECK"}

_lib = None
_lock = threading.Lock()

_vp, _i, _d, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t


class Sb2Error(RuntimeError):
    def __init__(self, fn: str, status: int):
        msg = lib().sb2_status_string(status).decode()
        super().__init__(f"{fn} failed: {STATUS.get(status, status)} ({msg})")
        self.status = status


class SystemDesc(ctypes.Structure):
    _fields_ = [("N", _i), ("T", _i), ("dt", _d), ("v", _vp), ("h", _vp), ("rho_hist", _vp), ("I_out", _vp)]


def lib() -> ctypes.CDLL:
    """Load libsb2.so once; raise if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1905_01180_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.sb2_status_string.restype = ctypes.c_char_p
        L.sb2_status_string.argtypes = [_i]
        L.sb2_version.restype = ctypes.c_char_p
        L.sb2_workspace_size.restype = _sz
        L.sb2_workspace_size.argtypes = [_i, _i, _i, _i]
        L.sb2_sigma.restype = _i
        L.sb2_sigma.argtypes = [_i, _i, _vp, _vp, _vp, _vp, _vp, _i, _vp, _sz, _vp]
        L.sb2_collision.restype = _i
        L.sb2_collision.argtypes = [_i, _i, _vp, _vp, _vp, _d, _vp, _vp, _i, _vp, _sz, _vp]
        L.sb2_collision_backward.restype = _i
        L.sb2_collision_backward.argtypes = [_i, _i, _vp, _vp, _vp, _d, _vp, _vp, _vp, _vp, _i, _vp, _sz, _vp]
        L.sb2_collision_batched.restype = _i
        L.sb2_collision_batched.argtypes = [_i, ctypes.POINTER(SystemDesc), _i, _vp, _sz, _vp]
        L.sb2_batched_workspace_size.restype = _sz
        L.sb2_batched_workspace_size.argtypes = [_i, ctypes.POINTER(SystemDesc), _i]
        L.sb2_autotune.restype = _i
        L.sb2_autotune.argtypes = [_i, _i, _vp, _vp, _vp, _d, _i, _vp, _sz, _vp, ctypes.POINTER(_i),
                                   ctypes.POINTER(_i), ctypes.POINTER(_i)]
        L.sb2_set_tuning.restype = _i
        L.sb2_set_tuning.argtypes = [_i, _i, _i, _i, _i]
        L.sb2_rho_step.restype = _i
        L.sb2_rho_step.argtypes = [_i, _vp, _vp, _vp, _d, _vp, _vp, _sz, _vp]
        L.sb2_collision_noalloc.restype = _i
        L.sb2_collision_noalloc.argtypes = [_i, _i, _vp, _vp, _vp, _d, _vp, _vp, _i, _vp]
        L.sb2_collision_v8.restype = _i
        L.sb2_collision_v8.argtypes = [_i, _i, _vp, _vp, _vp, _d, _vp, _vp, _i, _vp, _sz, _vp]
        L.sb2_collision_prop.restype = _i
        L.sb2_collision_prop.argtypes = [_i, _i, _vp, _vp, _vp, _d, _vp, _vp, _i, _vp, _sz, _vp]
        L.sb2_v8_count.restype = _sz
        L.sb2_v8_count.argtypes = [_i]
        L.sb2_v8_expand.restype = _i
        L.sb2_v8_expand.argtypes = [_i, _vp, _vp, _vp]
        L.sb2_collision_vertex.restype = _i
        L.sb2_collision_vertex.argtypes = [_i, _i, _i, _vp, _vp, _vp, _d, _vp, _vp, _vp, _sz, _vp]
        L.sb2_gkba_propagate_vertex.restype = _i
        L.sb2_gkba_propagate_vertex.argtypes = [_i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _d, _i, _vp, _sz, _vp]
        L.sb2_gkba_propagate_linear.restype = _i
        L.sb2_gkba_propagate_linear.argtypes = [_i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _d, _i, _vp, _sz,
                                                 _vp]
        L.sb2_gkba_propagate_qp.restype = _i
        L.sb2_gkba_propagate_qp.argtypes = [_i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _d, _i, _i, _vp, _sz, _vp]
        L.sb2_gkba_propagate_switched.restype = _i
        L.sb2_gkba_propagate_switched.argtypes = [_i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _d, _i, _i, _vp, _sz,
                                                  _vp]
        L.sb2_gkba_propagate.restype = _i
        L.sb2_gkba_propagate.argtypes = [_i, _i, _i, _vp, _vp, _vp, _vp, _vp, _d, _i, _i, _vp, _sz, _vp]
        _lib = L
        return L


def header_functions():
    """Names of the functions declared in include/sb2.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(sb2_\w+)\s*\(", txt, re.M)))


def _prec(prec) -> int:
    if isinstance(prec, int):
        return prec
    if prec not in PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}, got {prec!r}")
    return PRECISIONS[prec]


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


class WorkspaceCache:
    """Reusable device workspaces, one per (device, stream).

    Calls that share a workspace must be ordered on one stream, so the cache
    keys its buffers by the device index and the HIP stream the call is
    enqueued on: calls on two streams never share scratch memory.  Each use
    marks the buffer as in use on that stream (`record_stream`), so when an
    outgrown buffer is dropped the caching allocator does not hand its memory
    to other work before that stream has finished with it.  A buffer used
    while the stream was being captured into a HIP graph is never dropped on
    growth (the graph keeps its raw pointer and may be replayed later); it is
    retired and stays alive until `clear()`, which may only be called when no
    such graph will be replayed again.
    """

    def __init__(self, alloc=None):
        self._alloc = alloc or (lambda nbytes, dev: torch.empty(nbytes, dtype=torch.uint8, device=dev))
        self._bufs = {}
        self._captured = set()     # keys whose current buffer a graph capture used
        self._retired = []

    def get(self, nbytes: int, dev, key_dev: int, key_stream: int, stream=None, capturing: bool = False):
        key = (key_dev, key_stream)
        buf = self._bufs.get(key)
        if buf is None or buf.numel() < nbytes:
            if buf is not None and key in self._captured:
                self._retired.append(buf)
            self._captured.discard(key)
            buf = self._alloc(max(int(nbytes), 256), dev)
            self._bufs[key] = buf
        if capturing:
            self._captured.add(key)            # kept alive for replays; no stream bookkeeping under capture
        elif stream is not None and hasattr(buf, "record_stream"):
            buf.record_stream(stream)
        return buf

    def clear(self):
        self._bufs.clear()
        self._captured.clear()
        self._retired.clear()

    @property
    def retired(self):
        return len(self._retired)

    def __len__(self):
        return len(self._bufs)


_ws = WorkspaceCache()


def workspace(nbytes: int, dev: torch.device) -> torch.Tensor:
    """A cached device buffer of at least nbytes for the current stream of dev."""
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    st = torch.cuda.current_stream(idx)
    return _ws.get(nbytes, dev, idx, st.cuda_stream, st, torch.cuda.is_current_stream_capturing())


def release_workspace():
    """Free every cached workspace (including those outgrown); no captured
    graph that used them may be replayed afterwards."""
    _ws.clear()


def _check(t: torch.Tensor, name: str, dtype, shape):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _call(fn: str, *args):
    st = getattr(lib(), fn)(*args)
    if st != 0:
        raise Sb2Error(fn, st)


def sb2_workspace_size(op: str, n: int, t: int, prec="fp64") -> int:
    return int(lib().sb2_workspace_size(OPS[op] if isinstance(op, str) else op, n, t, _prec(prec)))


def sb2_sigma(v: torch.Tensor, g_less: torch.Tensor, g_great: torch.Tensor, prec="fp64"):
    """Sigma^<, Sigma^> (B, N, N) complex128 for B pairs G^<(t,t'_b), G^>(t,t'_b)."""
    b, n = g_less.shape[0], g_less.shape[1]
    _check(v, "v", torch.float64, (n, n, n, n))
    _check(g_less, "g_less", torch.complex128, (b, n, n))
    _check(g_great, "g_great", torch.complex128, (b, n, n))
    p = _prec(prec)
    nbytes = sb2_workspace_size("sigma", n, b, p)
    ws = workspace(nbytes, v.device)
    s_less = torch.empty_like(g_less)
    s_great = torch.empty_like(g_great)
    _call("sb2_sigma", n, b, v.data_ptr(), g_less.data_ptr(), g_great.data_ptr(), s_less.data_ptr(),
          s_great.data_ptr(), p, ws.data_ptr(), ws.numel(), _stream(v.device))
    return s_less, s_great


def sb2_collision(v: torch.Tensor, h: torch.Tensor, rho_hist: torch.Tensor, dt: float, prec="fp64",
                  return_sigma: bool = False):
    """I_ns(t) (N, N) complex128; with return_sigma also Sigma (2, T, N, N)."""
    t, n = rho_hist.shape[0], rho_hist.shape[1]
    _check(v, "v", torch.float64, (n, n, n, n))
    _check(h, "h", torch.complex128, (n, n))
    _check(rho_hist, "rho_hist", torch.complex128, (t, n, n))
    p = _prec(prec)
    ws = workspace(sb2_workspace_size("collision", n, t, p), v.device)
    out = torch.empty((n, n), dtype=torch.complex128, device=v.device)
    sig = torch.empty((2, t, n, n), dtype=torch.complex128, device=v.device) if return_sigma else None
    _call("sb2_collision", n, t, v.data_ptr(), h.data_ptr(), rho_hist.data_ptr(), float(dt), out.data_ptr(),
          sig.data_ptr() if sig is not None else None, p, ws.data_ptr(), ws.numel(), _stream(v.device))
    return (out, sig) if return_sigma else out


def sb2_collision_noalloc(v: torch.Tensor, h: torch.Tensor, rho_hist: torch.Tensor, dt: float, prec="fp64",
                          return_sigma: bool = False):
    """sb2_collision through the allocation-free entry point: the library's
    static per-device scratch buffer instead of a workspace (problems that do
    not fit it raise SB2_ESCRATCH)."""
    t, n = rho_hist.shape[0], rho_hist.shape[1]
    _check(v, "v", torch.float64, (n, n, n, n))
    _check(h, "h", torch.complex128, (n, n))
    _check(rho_hist, "rho_hist", torch.complex128, (t, n, n))
    p = _prec(prec)
    out = torch.empty((n, n), dtype=torch.complex128, device=v.device)
    sig = torch.empty((2, t, n, n), dtype=torch.complex128, device=v.device) if return_sigma else None
    _call("sb2_collision_noalloc", n, t, v.data_ptr(), h.data_ptr(), rho_hist.data_ptr(), float(dt),
          out.data_ptr(), sig.data_ptr() if sig is not None else None, p, _stream(v.device))
    return (out, sig) if return_sigma else out


def sb2_collision_prop(v: torch.Tensor, u_hist: torch.Tensor, rho_hist: torch.Tensor, dt: float, prec="fp64",
                       return_sigma: bool = False):
    """I_ns(t) (N, N) from given propagators u_hist[k] = U(t, t_k) (T, N, N)."""
    t, n = rho_hist.shape[0], rho_hist.shape[1]
    _check(v, "v", torch.float64, (n, n, n, n))
    _check(u_hist, "u_hist", torch.complex128, (t, n, n))
    _check(rho_hist, "rho_hist", torch.complex128, (t, n, n))
    p = _prec(prec)
    ws = workspace(sb2_workspace_size("collision", n, t, p), v.device)
    out = torch.empty((n, n), dtype=torch.complex128, device=v.device)
    sig = torch.empty((2, t, n, n), dtype=torch.complex128, device=v.device) if return_sigma else None
    _call("sb2_collision_prop", n, t, v.data_ptr(), u_hist.data_ptr(), rho_hist.data_ptr(), float(dt),
          out.data_ptr(), sig.data_ptr() if sig is not None else None, p, ws.data_ptr(), ws.numel(),
          _stream(v.device))
    return (out, sig) if return_sigma else out


def sb2_collision_v8(packed: torch.Tensor, h: torch.Tensor, rho_hist: torch.Tensor, dt: float, prec="fp64",
                     return_sigma: bool = False):
    """sb2_collision with v given as its 8-fold packed values (sb2_v8_count(N),)."""
    t, n = rho_hist.shape[0], rho_hist.shape[1]
    _check(packed, "packed", torch.float64, (int(lib().sb2_v8_count(n)),))
    _check(h, "h", torch.complex128, (n, n))
    _check(rho_hist, "rho_hist", torch.complex128, (t, n, n))
    p = _prec(prec)
    ws = workspace(sb2_workspace_size("collision", n, t, p), h.device)
    out = torch.empty((n, n), dtype=torch.complex128, device=h.device)
    sig = torch.empty((2, t, n, n), dtype=torch.complex128, device=h.device) if return_sigma else None
    _call("sb2_collision_v8", n, t, packed.data_ptr(), h.data_ptr(), rho_hist.data_ptr(), float(dt), out.data_ptr(),
          sig.data_ptr() if sig is not None else None, p, ws.data_ptr(), ws.numel(), _stream(h.device))
    return (out, sig) if return_sigma else out


def sb2_v8_expand(packed: torch.Tensor, n: int) -> torch.Tensor:
    """Full (N, N, N, N) float64 tensor from its 8-fold packed values (device)."""
    _check(packed, "packed", torch.float64, (int(lib().sb2_v8_count(n)),))
    v = torch.empty((n, n, n, n), dtype=torch.float64, device=packed.device)
    _call("sb2_v8_expand", n, packed.data_ptr(), v.data_ptr(), _stream(packed.device))
    return v


def sb2_collision_vertex(vertex: str, param: torch.Tensor, h: torch.Tensor, rho_hist: torch.Tensor, dt: float,
                         return_sigma: bool = False):
    """I_ns(t) (N, N) for a special vertex: 'diagonal' (param U, (N,)) or
    'symmetric' (param V, (N, N)); float64 throughout."""
    t, n = rho_hist.shape[0], rho_hist.shape[1]
    if vertex not in VERTICES:
        raise ValueError(f"vertex must be one of {sorted(VERTICES)}, got {vertex!r}")
    _check(param, "param", torch.float64, (n,) if vertex == "diagonal" else (n, n))
    _check(h, "h", torch.complex128, (n, n))
    _check(rho_hist, "rho_hist", torch.complex128, (t, n, n))
    ws = workspace(sb2_workspace_size("collision_" + vertex, n, t, 0), h.device)
    out = torch.empty((n, n), dtype=torch.complex128, device=h.device)
    sig = torch.empty((2, t, n, n), dtype=torch.complex128, device=h.device) if return_sigma else None
    _call("sb2_collision_vertex", n, t, VERTICES[vertex], param.data_ptr(), h.data_ptr(), rho_hist.data_ptr(),
          float(dt), out.data_ptr(), sig.data_ptr() if sig is not None else None, ws.data_ptr(), ws.numel(),
          _stream(h.device))
    return (out, sig) if return_sigma else out


def sb2_gkba_propagate(v, h, rho_hist, u_hist, n0: int, nsteps: int, dt: float, prec="fp64", hf: bool = True,
                       collision: bool = True, i_hist=None, switch=None, sigma_qp=None):
    """Advance the propagation state in place from step n0 to n0 + nsteps.

    rho_hist (C, N, N) with C >= n0 + nsteps + 1, u_hist and i_hist (C', N, N)
    with C' >= n0 + nsteps (i_hist optional); all complex128 on the device.
    switch: optional device float64 coupling history lambda(t_m) (the
    interaction is lambda(t) v; sb2_gkba_propagate_switched).
    sigma_qp: optional constant (N, N) complex128 correction of the GKBA
    propagators (sb2_gkba_propagate_qp); not combined with switch.
    """
    n = h.shape[0]
    _check(v, "v", torch.float64, (n, n, n, n))
    _check(h, "h", torch.complex128, (n, n))
    _check(rho_hist, "rho_hist", torch.complex128, (rho_hist.shape[0], n, n))
    _check(u_hist, "u_hist", torch.complex128, (u_hist.shape[0], n, n))
    if rho_hist.shape[0] < n0 + nsteps + 1 or u_hist.shape[0] < max(n0 + nsteps, 1):
        raise ValueError("rho_hist / u_hist capacity too small for n0 + nsteps")
    if i_hist is not None:
        _check(i_hist, "i_hist", torch.complex128, (i_hist.shape[0], n, n))
        if i_hist.shape[0] < n0 + nsteps:
            raise ValueError("i_hist capacity too small for n0 + nsteps")
    p = _prec(prec)
    ws = workspace(sb2_workspace_size("propagate", n, n0 + nsteps, p), v.device)
    flags = (PROP_HF if hf else 0) | (PROP_COLLISION if collision else 0)
    if switch is not None and sigma_qp is not None:
        raise ValueError("switch and sigma_qp are separate entry points; pass one of them")
    if sigma_qp is not None:
        _check(sigma_qp, "sigma_qp", torch.complex128, (n, n))
        _call("sb2_gkba_propagate_qp", n, int(n0), int(nsteps), v.data_ptr(), h.data_ptr(), sigma_qp.data_ptr(),
              rho_hist.data_ptr(), u_hist.data_ptr(), i_hist.data_ptr() if i_hist is not None else None,
              float(dt), flags, p, ws.data_ptr(), ws.numel(), _stream(v.device))
        return
    if switch is not None:
        # time-dependent coupling: switch[m] = lambda(t_m), m < n0 + nsteps (device float64)
        _check(switch, "switch", torch.float64, (switch.shape[0],))
        if switch.shape[0] < n0 + nsteps:
            raise ValueError("switch must hold lambda(t_m) for every m < n0 + nsteps")
        _call("sb2_gkba_propagate_switched", n, int(n0), int(nsteps), v.data_ptr(), h.data_ptr(),
              rho_hist.data_ptr(), u_hist.data_ptr(), i_hist.data_ptr() if i_hist is not None else None,
              switch.data_ptr(), float(dt), flags, p, ws.data_ptr(), ws.numel(), _stream(v.device))
        return
    _call("sb2_gkba_propagate", n, int(n0), int(nsteps), v.data_ptr(), h.data_ptr(), rho_hist.data_ptr(),
          u_hist.data_ptr(), i_hist.data_ptr() if i_hist is not None else None, float(dt), flags, p,
          ws.data_ptr(), ws.numel(), _stream(v.device))


def sb2_gkba_propagate_linear(v, h, rho_hist, p_state, m_state, n0: int, nsteps: int, dt: float, hf: bool = True,
                              collision: bool = True, i_hist=None, switch=None):
    """sb2_gkba_propagate with the sum over past times carried in the state
    (p_state (N, N) = U(t_n, t_0), m_state (N^4,) the accumulated tensor),
    float64; rho_hist (and i_hist) as for sb2_gkba_propagate, advanced in
    place; at n0 = 0 the call initialises p_state and m_state.  switch:
    optional device float64 coupling history lambda(t_m), m < n0 + nsteps."""
    n = h.shape[0]
    _check(v, "v", torch.float64, (n, n, n, n))
    _check(h, "h", torch.complex128, (n, n))
    _check(rho_hist, "rho_hist", torch.complex128, (rho_hist.shape[0], n, n))
    _check(p_state, "p_state", torch.complex128, (n, n))
    _check(m_state, "m_state", torch.complex128, (n ** 4,))
    if rho_hist.shape[0] < n0 + nsteps + 1:
        raise ValueError("rho_hist capacity too small for n0 + nsteps")
    if i_hist is not None:
        _check(i_hist, "i_hist", torch.complex128, (i_hist.shape[0], n, n))
        if i_hist.shape[0] < n0 + nsteps:
            raise ValueError("i_hist capacity too small for n0 + nsteps")
    if switch is not None:
        _check(switch, "switch", torch.float64, (switch.shape[0],))
        if switch.shape[0] < n0 + nsteps:
            raise ValueError("switch must hold lambda(t_m) for every m < n0 + nsteps")
    ws = workspace(sb2_workspace_size("propagate_linear", n, 1, 0), v.device)
    flags = (PROP_HF if hf else 0) | (PROP_COLLISION if collision else 0)
    _call("sb2_gkba_propagate_linear", n, int(n0), int(nsteps), v.data_ptr(), h.data_ptr(), rho_hist.data_ptr(),
          p_state.data_ptr(), m_state.data_ptr(), i_hist.data_ptr() if i_hist is not None else None,
          switch.data_ptr() if switch is not None else None, float(dt), flags, ws.data_ptr(), ws.numel(),
          _stream(v.device))


def sb2_gkba_propagate_vertex(vertex: str, param, h, rho_hist, u_hist, n0: int, nsteps: int, dt: float,
                              hf: bool = True, collision: bool = True, i_hist=None):
    """sb2_gkba_propagate for a special vertex ('diagonal': param U (N,),
    'symmetric': param V (N, N)), float64; state arrays as for
    sb2_gkba_propagate, advanced in place."""
    n = h.shape[0]
    if vertex not in VERTICES:
        raise ValueError(f"vertex must be one of {sorted(VERTICES)}, got {vertex!r}")
    _check(param, "param", torch.float64, (n,) if vertex == "diagonal" else (n, n))
    _check(h, "h", torch.complex128, (n, n))
    _check(rho_hist, "rho_hist", torch.complex128, (rho_hist.shape[0], n, n))
    _check(u_hist, "u_hist", torch.complex128, (u_hist.shape[0], n, n))
    if rho_hist.shape[0] < n0 + nsteps + 1 or u_hist.shape[0] < max(n0 + nsteps, 1):
        raise ValueError("rho_hist / u_hist capacity too small for n0 + nsteps")
    if i_hist is not None:
        _check(i_hist, "i_hist", torch.complex128, (i_hist.shape[0], n, n))
        if i_hist.shape[0] < n0 + nsteps:
            raise ValueError("i_hist capacity too small for n0 + nsteps")
    ws = workspace(sb2_workspace_size("propagate_" + vertex, n, n0 + nsteps, 0), h.device)
    flags = (PROP_HF if hf else 0) | (PROP_COLLISION if collision else 0)
    _call("sb2_gkba_propagate_vertex", n, int(n0), int(nsteps), VERTICES[vertex], param.data_ptr(), h.data_ptr(),
          rho_hist.data_ptr(), u_hist.data_ptr(), i_hist.data_ptr() if i_hist is not None else None, float(dt),
          flags, ws.data_ptr(), ws.numel(), _stream(h.device))


def sb2_collision_backward(v, h, rho_hist, dt, grad_i, prec="fp64"):
    """(dL/dv, dL/dh, dL/drho_hist) for the cotangent grad_i = dL/dI (torch convention)."""
    t, n = rho_hist.shape[0], rho_hist.shape[1]
    _check(v, "v", torch.float64, (n, n, n, n))
    _check(h, "h", torch.complex128, (n, n))
    _check(rho_hist, "rho_hist", torch.complex128, (t, n, n))
    _check(grad_i, "grad_i", torch.complex128, (n, n))
    p = _prec(prec)
    ws = workspace(sb2_workspace_size("collision_backward", n, t, p), v.device)
    gv = torch.empty_like(v)
    gh = torch.empty_like(h)
    gr = torch.empty_like(rho_hist)
    _call("sb2_collision_backward", n, t, v.data_ptr(), h.data_ptr(), rho_hist.data_ptr(), float(dt),
          grad_i.data_ptr(), gv.data_ptr(), gh.data_ptr(), gr.data_ptr(), p, ws.data_ptr(), ws.numel(),
          _stream(v.device))
    return gv, gh, gr


def sb2_rho_step(h, rho, i_ns, dt):
    """rho(t+dt) = U rho U^dag - dt (I + I^dag), U = exp(-i h dt)."""
    n = h.shape[0]
    for name, x in (("h", h), ("rho", rho), ("i_ns", i_ns)):
        _check(x, name, torch.complex128, (n, n))
    ws = workspace(sb2_workspace_size("rho_step", n, 1, 0), h.device)
    out = torch.empty_like(rho)
    _call("sb2_rho_step", n, h.data_ptr(), rho.data_ptr(), i_ns.data_ptr(), float(dt), out.data_ptr(),
          ws.data_ptr(), ws.numel(), _stream(h.device))
    return out


def _descs(systems, outs):
    arr = (SystemDesc * len(systems))()
    for d, (v, h, rho, dt), o in zip(arr, systems, outs):
        n, t = h.shape[0], rho.shape[0]
        _check(v, "v", torch.float64, (n, n, n, n))
        _check(h, "h", torch.complex128, (n, n))
        _check(rho, "rho_hist", torch.complex128, (t, n, n))
        d.N, d.T, d.dt = n, t, float(dt)
        d.v, d.h, d.rho_hist, d.I_out = v.data_ptr(), h.data_ptr(), rho.data_ptr(), o.data_ptr()
    return arr


def sb2_collision_batched(systems, prec="fp16x3"):
    """I_ns for a list of (v, h, rho_hist, dt) systems in one enqueue."""
    outs = [torch.empty((h.shape[0], h.shape[0]), dtype=torch.complex128, device=h.device)
            for (_, h, _, _) in systems]
    arr = _descs(systems, outs)
    p = _prec(prec)
    dev = systems[0][1].device
    nbytes = int(lib().sb2_batched_workspace_size(len(systems), arr, p))
    ws = workspace(nbytes, dev)
    _call("sb2_collision_batched", len(systems), arr, p, ws.data_ptr(), ws.numel(), _stream(dev))
    return outs


def sb2_autotune(v, h, rho_hist, dt, prec="fp16x3"):
    """Tune the launch parameters for (N, prec) on this workload's first chunk.

    Returns {"persist": workgroups per single-slab launch, "r4pct": split-K
    factor of the last contraction in percent, "fused": workgroups of the fused
    second/third contraction (0 = separate launches)}; the library keeps the
    values for later calls in this process."""
    t, n = rho_hist.shape[0], rho_hist.shape[1]
    _check(v, "v", torch.float64, (n, n, n, n))
    _check(h, "h", torch.complex128, (n, n))
    _check(rho_hist, "rho_hist", torch.complex128, (t, n, n))
    p = _prec(prec)
    ws = workspace(sb2_workspace_size("autotune", n, t, p), v.device)
    persist, r4pct, fused = _i(0), _i(0), _i(0)
    _call("sb2_autotune", n, t, v.data_ptr(), h.data_ptr(), rho_hist.data_ptr(), float(dt), p, ws.data_ptr(),
          ws.numel(), _stream(v.device), ctypes.byref(persist), ctypes.byref(r4pct), ctypes.byref(fused))
    return {"persist": persist.value, "r4pct": r4pct.value, "fused": fused.value}


DEFAULT_TUNING = {"persist": 768, "r4pct": 100, "fused": 512}
DEFAULT_PERSIST_FP16X3 = 3072          # the library's default for split float16


def sb2_set_tuning(n: int, prec, persist: int = None, r4pct: int = 100, fused: int = 512):
    """Install launch parameters for (n, prec), e.g. from an earlier
    sb2_autotune; persist=None takes the library's default for prec."""
    p = _prec(prec)
    if persist is None:
        persist = DEFAULT_PERSIST_FP16X3 if p == PRECISIONS["fp16x3"] else DEFAULT_TUNING["persist"]
    _call("sb2_set_tuning", n, p, persist, r4pct, fused)
