"""Symmetries of the seeded interaction tensors (inputs.py), as documented:
the low-rank construction has {ijkl, jilk, klij, lkji} plus i <-> j alone
(so its exchange term is exactly -1/2 of the direct one), the real-orbital
construction has exactly the 8-fold group of Eq. 4 and not i <-> j, the
group-averaged one has the four-element group only."""
import numpy as np

from oracle import sb2_oracle as o
from paper_1905_01180_amd import inputs as gen

EQ4 = [(0, 1, 2, 3), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0), (0, 2, 1, 3), (3, 1, 2, 0), (2, 0, 3, 1),
       (1, 3, 0, 2)]
FOUR = EQ4[:4]


def _sym(v, perm):
    return np.abs(v - v.transpose(perm)).max()


def test_lowrank_has_extra_pair_symmetry():
    v = gen.interaction_lowrank(6, np.random.default_rng(1))
    for p in FOUR:
        assert _sym(v, p) < 1e-15
    assert _sym(v, (1, 0, 2, 3)) < 1e-15            # i <-> j alone: not a symmetry of Eq. 4
    assert _sym(v, (0, 2, 1, 3)) > 1e-3             # but not the rest of Eq. 4's group
    # consequence: w = 2 v - v_qmsj = v, so Sigma = S_direct / 2 exactly
    g = np.random.default_rng(2)
    gm = g.standard_normal((6, 6)) + 1j * g.standard_normal((6, 6))
    gb = g.standard_normal((6, 6)) + 1j * g.standard_normal((6, 6))
    assert np.abs(o.exchange_combined(v) - v).max() < 1e-15
    s = o.sigma(v, gm, gb)
    direct = np.einsum("irpn,mqsj,nm,sr,pq->ij", v, v, gm, gb, gm)
    assert np.abs(s - direct).max() < 1e-12 * np.abs(direct).max()


def test_real_orbitals_have_exactly_eq4():
    v = gen.interaction_real_orbitals(6, np.random.default_rng(3))
    for p in EQ4:
        assert _sym(v, p) < 1e-14
    assert _sym(v, (1, 0, 2, 3)) > 1e-3


def test_generic_has_the_four_element_group_only():
    v = gen.interaction_generic(5, np.random.default_rng(4))
    for p in FOUR:
        assert _sym(v, p) < 1e-15
    for p in EQ4[4:] + [(1, 0, 2, 3)]:
        assert _sym(v, p) > 1e-3


def test_make_system_kinds():
    for kind in ("lowrank", "generic", "orbitals"):
        s = gen.make_system(4, 2, config_id=50, v_kind=kind)
        assert s.v.shape == (4, 4, 4, 4) and abs(np.abs(s.v).max() - 0.5) < 1e-15
