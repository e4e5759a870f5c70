"""8-fold packed interaction tensor: the format against brute-force orbits of
the symmetry group of Eq. 4 (host), and the library's expansion (GPU)."""
import itertools

import numpy as np
import pytest

from paper_1905_01180_amd import _lib
from paper_1905_01180_amd import inputs as gen
from paper_1905_01180_amd import v8

FAKE = 0x1000


def _images(i, j, k, l):
    # the eight index orders of Eq. 4 that leave a real Coulomb integral unchanged
    return {(i, j, k, l), (j, i, l, k), (k, l, i, j), (l, k, j, i),
            (i, k, j, l), (l, j, k, i), (k, i, l, j), (j, l, i, k)}


def _pair(a, b):
    return max(a, b) * (max(a, b) + 1) // 2 + min(a, b)


def _index(i, j, k, l):
    return _pair(_pair(i, l), _pair(j, k))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_orbit_count_and_index_invariance(n):
    orbits = set()
    for t in itertools.product(range(n), repeat=4):
        imgs = _images(*t)
        orbits.add(min(imgs))
        assert len({_index(*x) for x in imgs}) == 1           # one packed slot per orbit
    assert len(orbits) == v8.count(n) == _lib.lib().sb2_v8_count(n)
    # distinct orbits get distinct slots, and every slot is used
    assert sorted(_index(*o) for o in orbits) == list(range(v8.count(n)))


def test_pack_then_loop_unpack_reproduces_v():
    n = 6
    v = gen.interaction_real_orbitals(n, np.random.default_rng(1))
    assert v8.symmetry_error(v) < 1e-15
    p = v8.pack(v)
    assert p.shape == (v8.count(n),)
    for t in itertools.product(range(n), repeat=4):
        assert abs(p[_index(*t)] - v[t]) < 1e-15


def test_generators_symmetry():
    g = np.random.default_rng(2)
    assert v8.symmetry_error(gen.interaction_real_orbitals(7, g)) < 1e-15
    # the 4-element group of the low-rank generator is not the full group
    assert v8.symmetry_error(gen.interaction_lowrank(7, g)) > 1e-3


def test_abi_sizes_and_errors():
    L = _lib.lib()
    assert L.sb2_v8_count(0) == 0 and L.sb2_v8_count(129) == 0
    assert L.sb2_v8_count(100) == v8.count(100) == 12753775
    assert L.sb2_v8_expand(0, FAKE, FAKE, None) == -2
    assert L.sb2_v8_expand(5, None, FAKE, None) == -1
    assert L.sb2_v8_expand(5, FAKE, None, None) == -1


@pytest.mark.gpu
@pytest.mark.parametrize("n", [1, 2, 9, 64, 128])
def test_gpu_expand_is_exact(n):
    import torch
    dev = torch.device("cuda:0")
    v = gen.interaction_real_orbitals(n, np.random.default_rng(3 + n))
    p = v8.pack(v)
    got = _lib.sb2_v8_expand(torch.from_numpy(p).to(dev), n).cpu().numpy()
    rng = np.random.default_rng(n)
    idx = rng.integers(0, n, size=(20000, 4)) if n > 16 else np.array(list(itertools.product(range(n), repeat=4)))
    for t in idx:
        assert got[tuple(t)] == p[_index(*t)]                  # bit for bit
    # the expansion is exactly symmetric; v itself only to its rounding (an orbit
    # representative is at most three generator steps from any member)
    assert np.abs(got - v).max() <= 3.0 * v8.symmetry_error(v) + 1e-300


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x3"])
@pytest.mark.parametrize("n,t", [(1, 2), (5, 3), (17, 4), (33, 3), (100, 2), (120, 2)])
def test_gpu_packed_collision_is_bitwise_dense(n, t, prec):
    # the layout kernels read the packed values directly; the result must be
    # bit for bit the dense path's on the expanded tensor
    import torch
    from paper_1905_01180_amd import _lib
    s = gen.make_system(n, t, config_id=240, system_id=n, v_kind="orbitals")
    packed = torch.from_numpy(v8.pack(s.v)).to("cuda")
    h, r = torch.from_numpy(s.h).to("cuda"), torch.from_numpy(s.rho_hist).to("cuda")
    print(f"case: packed collision N={n} T={t} {prec}", flush=True)
    got, gsig = _lib.sb2_collision_v8(packed, h, r, s.dt, prec, return_sigma=True)
    dense = _lib.sb2_v8_expand(packed, n)
    want, wsig = _lib.sb2_collision(dense, h, r, s.dt, prec, return_sigma=True)
    torch.cuda.synchronize()
    assert torch.equal(got, want) and torch.equal(gsig, wsig)
    if n <= 33:
        # and the oracle's self-energies (I itself cancels to rounding noise at N = 1)
        from oracle import sb2_oracle as o
        _, ref = o.collision(s.v, s.h, s.rho_hist, s.dt, return_sigma=True)
        tol = 1e-11 if prec == "fp64" else 2e-6
        gsig = gsig.cpu().numpy()
        for k in range(t):
            for kind in (0, 1):
                assert np.abs(gsig[kind, k] - ref[k][kind]).max() < tol * np.abs(ref[k][kind]).max()
