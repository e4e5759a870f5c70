"""8-fold packed storage of a real interaction tensor (host side).

For real basis functions the Coulomb integrals (Eq. 3) obey the 8-point
symmetry of Eq. 4: v_ijkl depends only on the unordered pairs {i, l} and
{j, k} and is unchanged when the two pairs are exchanged, so about N^4 / 8
values determine it.  Packed index (the same as the library's
sb2_v8_expand):
    pair(a, b) = max(a,b) (max(a,b) + 1) / 2 + min(a,b)
    packed[pair(pair(i, l), pair(j, k))] = v_ijkl
pack() reads one representative per orbit; expansion to the full tensor runs
on the device (_lib.sb2_v8_expand).
"""
from __future__ import annotations

import numpy as np


def count(n: int) -> int:
    p = n * (n + 1) // 2
    return p * (p + 1) // 2


def _pairs(n: int):
    """(a, b) with a >= b for pair index 0 .. n(n+1)/2 - 1, in index order."""
    a, b = np.tril_indices(n)
    return a, b                     # row-major lower triangle: index a(a+1)/2 + b


def pack(v: np.ndarray) -> np.ndarray:
    """Packed float64 values of a real (n, n, n, n) tensor with the 8-point symmetry."""
    n = v.shape[0]
    if v.shape != (n, n, n, n):
        raise ValueError(f"v must be (n, n, n, n), got {v.shape}")
    pa, pb = _pairs(n)
    hi, lo = np.tril_indices(pa.shape[0])            # pair-of-pairs P >= Q, index P(P+1)/2 + Q
    i, l = pa[hi], pb[hi]                            # pair P = {i, l}
    j, k = pa[lo], pb[lo]                            # pair Q = {j, k}
    return np.ascontiguousarray(v[i, j, k, l], dtype=np.float64)


def symmetry_error(v: np.ndarray) -> float:
    """max |v_ijkl - v_g(ijkl)| over the generators of the 8-point group."""
    return max(float(np.abs(v - v.transpose(3, 1, 2, 0)).max()),   # i <-> l
               float(np.abs(v - v.transpose(0, 2, 1, 3)).max()),   # j <-> k
               float(np.abs(v - v.transpose(1, 0, 3, 2)).max()))   # (i,l) <-> (j,k): v_jilk
