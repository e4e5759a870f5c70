"""Policy of the binding's workspace cache (CPU only: a host allocator stands
in for device memory).  Calls on different streams must never share scratch
memory, an outgrown buffer that a graph capture used must stay alive for that
graph's replays, and one that no capture used is dropped."""
import torch

from paper_1905_01180_amd._lib import WorkspaceCache


def _cache():
    allocs = []

    def alloc(nbytes, dev):
        t = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        allocs.append(t)
        return t
    return WorkspaceCache(alloc), allocs


def test_one_buffer_per_device_and_stream():
    c, allocs = _cache()
    a = c.get(1000, "cpu", 0, 11)
    b = c.get(1000, "cpu", 0, 22)
    d = c.get(1000, "cpu", 1, 11)
    assert a.data_ptr() != b.data_ptr() and a.data_ptr() != d.data_ptr() and b.data_ptr() != d.data_ptr()
    assert len(c) == 3 and len(allocs) == 3
    # reuse on the same (device, stream), also for a smaller request
    assert c.get(500, "cpu", 0, 11).data_ptr() == a.data_ptr()
    assert len(allocs) == 3


def test_growth_drops_uncaptured_and_retires_captured():
    c, allocs = _cache()
    a = c.get(1000, "cpu", 0, 11)
    b = c.get(2000, "cpu", 0, 11)               # outgrown, never captured: dropped
    assert b.numel() >= 2000 and b.data_ptr() != a.data_ptr()
    assert c.retired == 0
    g = c.get(2000, "cpu", 0, 33, capturing=True)   # used by a capture
    g2 = c.get(4000, "cpu", 0, 33)                  # outgrown later: must survive
    assert c.retired == 1 and g2.numel() >= 4000
    assert g.data_ptr() != g2.data_ptr()
    # the new buffer was not captured: growing again drops it
    c.get(8000, "cpu", 0, 33)
    assert c.retired == 1
    c.clear()
    assert c.retired == 0 and len(c) == 0


def test_minimum_size():
    c, _ = _cache()
    assert c.get(0, "cpu", 0, 0).numel() == 256
