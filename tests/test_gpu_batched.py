"""Batched multi-system evaluation (sb2_collision_batched): every system's
I(t) against the FP64 oracle and against a single-system call, uneven N and T
(several 16-wide tiles, ragged tails), and replay of a captured HIP graph
against the eager result (several replays with eager work in between)."""
import numpy as np
import pytest

from oracle import sb2_oracle as o
from paper_1905_01180_amd import inputs as gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = [(3, 5), (17, 9), (24, 12), (40, 3), (33, 20), (1, 4)]
TOL = {"fp64": 1e-11, "fp32": 2e-6, "fp16x3": 2e-6}


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _systems(shapes):
    dev = torch.device("cuda")
    out = []
    for i, (n, t) in enumerate(shapes):
        s = gen.make_system(n, t, config_id=400, system_id=i)
        out.append((s, (torch.from_numpy(s.v).to(dev), torch.from_numpy(s.h).to(dev),
                        torch.from_numpy(s.rho_hist).to(dev), s.dt)))
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x3"])
def test_batched_against_oracle_and_single(prec):
    from paper_1905_01180_amd import _lib
    sy = _systems(SHAPES)
    print("case: batched", prec, SHAPES, flush=True)
    outs = _lib.sb2_collision_batched([d for _, d in sy], prec)
    torch.cuda.synchronize()
    for (s, d), got in zip(sy, outs):
        want = o.collision(s.v, s.h, s.rho_hist, s.dt)
        single = _lib.sb2_collision(*d, prec)
        g = got.cpu().numpy()
        assert rel(g, want) < TOL[prec] or np.abs(want).max() < 1e-14, (s.n, s.t, rel(g, want))
        assert rel(g, single.cpu().numpy()) < TOL[prec] or np.abs(want).max() < 1e-14


def test_batched_graph_replay_matches_eager():
    from paper_1905_01180_amd import _lib
    sy = _systems(SHAPES[:4])
    systems = [d for _, d in sy]
    print("case: batched graph replay", flush=True)
    eager = [x.clone() for x in _lib.sb2_collision_batched(systems, "fp16x3")]
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        _lib.sb2_collision_batched(systems, "fp16x3")          # warm the workspace outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        outs = _lib.sb2_collision_batched(systems, "fp16x3")
    for rep in range(3):
        for o_ in outs:
            o_.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs, eager):
            assert torch.equal(a, b), rep
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()   # eager work between replays


@pytest.mark.parametrize("prec", ["fp64", "fp16x3"])
def test_batched_mixed_solo_and_grouped(prec):
    """A system with at least 1e12 flops of contraction work (here N = 64,
    T = 20) runs on its own chain inside the batched call, the small ones in
    grouped rounds; the small ones match the oracle and every result matches
    the single-system call (itself checked against the oracle elsewhere)."""
    from paper_1905_01180_amd import _lib
    shapes = [(64, 20), (20, 5), (9, 4), (37, 3)]
    assert 48 * 20 * 64 ** 5 >= 1e12 and all(48 * t * n ** 5 < 1e12 for n, t in shapes[1:])
    sy = _systems(shapes)
    print("case: batched mixed", prec, shapes, flush=True)
    outs = _lib.sb2_collision_batched([d for _, d in sy], prec)
    torch.cuda.synchronize()
    for (s, d), got in zip(sy, outs):
        g = got.cpu().numpy()
        single = _lib.sb2_collision(*d, prec).cpu().numpy()
        assert rel(g, single) < TOL[prec], (s.n, s.t, rel(g, single))
        if s.n < 64:
            want = o.collision(s.v, s.h, s.rho_hist, s.dt)
            assert rel(g, want) < TOL[prec], (s.n, s.t, rel(g, want))
