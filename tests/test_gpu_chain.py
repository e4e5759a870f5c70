"""GKBA propagation with the special vertices of Sec. III on the device
(sb2_gkba_propagate_vertex) against the propagation oracle run with the
materialised vertex tensor (oracle/gkba_driver.py with v_ijkl built from U or
V): the paper's chains of Sec. IV (N_b = 10 sites, hopping J = -1, U = 1,
Ohno V_ij = U / sqrt(1 + |i - j|^2), the left half filled at t = 0) for the
first 120 / 80 steps of their runs, random vertices with every combination of
terms, and the general-vertex device propagation with the same tensor.
Bars: float64, 1e-11 relative (Frobenius) on every rho and I."""
import numpy as np
import pytest

from oracle import gkba_driver as d
from oracle import sb2_oracle as o
from paper_1905_01180_amd import inputs as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def relf(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def run_vertex(vertex, param, h, rho0, dt, steps, hf=True, coll=True):
    from paper_1905_01180_amd import _lib
    n = h.shape[0]
    rho = torch.zeros((steps + 1, n, n), dtype=torch.complex128, device=DEV)
    u = torch.zeros((steps, n, n), dtype=torch.complex128, device=DEV)
    ih = torch.zeros((steps, n, n), dtype=torch.complex128, device=DEV)
    rho[0].copy_(_dev(rho0))
    _lib.sb2_gkba_propagate_vertex(vertex, _dev(param), _dev(h), rho, u, 0, steps, dt, hf=hf, collision=coll,
                                   i_hist=ih)
    return rho.cpu().numpy(), u.cpu().numpy(), ih.cpu().numpy()


def tensor(vertex, param):
    return o.vertex_diagonal(param) if vertex == "diagonal" else o.vertex_symmetric(param)


@pytest.mark.parametrize("vertex,dt,steps", [("diagonal", 0.01, 120), ("symmetric", 0.025, 80)])
def test_paper_chains_match_oracle(vertex, dt, steps):
    n = 10
    h = gen.chain_hopping(n, -1.0)
    param = gen.hubbard_onsite(n, 1.0) if vertex == "diagonal" else gen.ohno_matrix(n, 1.0)
    rho0 = gen.left_half_density(n)
    print(f"case: {vertex} chain N={n} dt={dt} steps={steps}", flush=True)
    rho, u, ih = run_vertex(vertex, param, h, rho0, dt, steps)
    ref = d.propagate(tensor(vertex, param), h, dt, steps, d.new_state(rho0))
    e_rho = max(relf(rho[m], ref["rho"][m]) for m in range(steps + 1))
    e_i = max(relf(ih[m], ref["i"][m]) for m in range(1, steps))
    e_u = max(relf(u[k], ref["u"][k]) for k in range(steps))
    print(f"{vertex} chain: rho {e_rho:.2e}, I {e_i:.2e}, U {e_u:.2e}", flush=True)
    assert e_rho < 1e-11 and e_i < 1e-11 and e_u < 1e-11
    # the density leaves the left half and keeps its trace
    assert np.real(np.trace(rho[-1][n // 2:, n // 2:])) > 0.05
    assert abs(np.trace(rho[-1]) - n // 2) < 1e-11


@pytest.mark.parametrize("hf,coll", [(True, True), (False, True), (True, False)])
@pytest.mark.parametrize("vertex,n", [("diagonal", 7), ("symmetric", 13)])
def test_random_vertex_propagation(vertex, n, hf, coll):
    g = np.random.default_rng(300 + n)
    h = gen.hermitian_gaussian(n, g)
    param = g.uniform(0.2, 1.0, n) if vertex == "diagonal" else gen.ohno_matrix(n, 0.8) * g.uniform(0.5, 1.0, (n, n))
    if vertex == "symmetric":
        param = 0.5 * (param + param.T)
    rho0 = gen.density_matrix(n, g)
    steps, dt = 8, 0.05
    print(f"case: {vertex} N={n} hf={hf} coll={coll}", flush=True)
    rho, _, ih = run_vertex(vertex, param, h, rho0, dt, steps, hf, coll)
    ref = d.propagate(tensor(vertex, param), h, dt, steps, d.new_state(rho0), hf=hf, collision=coll)
    e_rho = max(relf(rho[m], ref["rho"][m]) for m in range(steps + 1))
    print(f"{vertex} N={n} hf={hf} coll={coll}: rho {e_rho:.2e}", flush=True)
    assert e_rho < 1e-11
    if coll:
        assert max(relf(ih[m], ref["i"][m]) for m in range(1, steps)) < 1e-11
    else:
        assert np.abs(ih).max() == 0.0


@pytest.mark.parametrize("vertex", ["diagonal", "symmetric"])
def test_vertex_equals_general_propagation(vertex):
    from paper_1905_01180_amd import _lib
    n, steps, dt = 10, 30, 0.025
    h = gen.chain_hopping(n, -1.0)
    param = gen.hubbard_onsite(n, 1.0) if vertex == "diagonal" else gen.ohno_matrix(n, 1.0)
    rho0 = gen.left_half_density(n)
    print(f"case: {vertex} vs general N={n}", flush=True)
    rho_v, _, _ = run_vertex(vertex, param, h, rho0, dt, steps)
    rho = torch.zeros((steps + 1, n, n), dtype=torch.complex128, device=DEV)
    u = torch.zeros((steps, n, n), dtype=torch.complex128, device=DEV)
    rho[0].copy_(_dev(rho0))
    _lib.sb2_gkba_propagate(_dev(tensor(vertex, param)), _dev(h), rho, u, 0, steps, dt, "fp64")
    rho = rho.cpu().numpy()
    assert max(relf(rho_v[m], rho[m]) for m in range(steps + 1)) < 1e-12
