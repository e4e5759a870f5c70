"""Host-side checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments before enqueueing anything (these
calls never reach the GPU, so they run on the CPU-only container)."""
import ctypes

import pytest

from paper_1905_01180_amd import _lib


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def test_exports_every_header_function(L):
    names = _lib.header_functions()
    assert {"sb2_sigma", "sb2_collision", "sb2_collision_backward", "sb2_collision_batched",
            "sb2_rho_step", "sb2_workspace_size", "sb2_status_string"} <= set(names)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    for code in (0, -1, -2, -3, -4, -5):
        assert len(L.sb2_status_string(code)) > 0
    assert L.sb2_status_string(12345) == b"unknown status"


def test_workspace_sizes(L):
    ws = _lib.sb2_workspace_size
    assert ws("collision", 0, 10, "fp64") == 0
    assert ws("collision", 129, 10, "fp64") == 0
    assert ws("collision", 10, 0, "fp64") == 0
    assert ws("collision", 10, 10, 7) == 0
    a = ws("collision", 10, 20, "fp64")
    b = ws("collision", 10, 40, "fp64")
    assert 0 < a < b
    assert ws("sigma", 12, 3, "fp32") > 0
    assert ws("rho_step", 12, 1, "fp64") > 0
    assert a % 256 == 0


FAKE = 0x1000   # never dereferenced: validation fails first


def test_argument_errors_are_reported_before_enqueue(L):
    big = 1 << 40
    c = L.sb2_collision
    # shape errors
    assert c(0, 10, FAKE, FAKE, FAKE, 0.05, FAKE, None, 0, FAKE, big, None) == -2
    assert c(10, 0, FAKE, FAKE, FAKE, 0.05, FAKE, None, 0, FAKE, big, None) == -2
    assert c(200, 10, FAKE, FAKE, FAKE, 0.05, FAKE, None, 0, FAKE, big, None) == -2
    # invalid arguments
    assert c(10, 10, None, FAKE, FAKE, 0.05, FAKE, None, 0, FAKE, big, None) == -1
    assert c(10, 10, FAKE, FAKE, FAKE, float("nan"), FAKE, None, 0, FAKE, big, None) == -1
    assert c(10, 10, FAKE, FAKE, FAKE, -0.05, FAKE, None, 0, FAKE, big, None) == -1
    assert c(10, 10, FAKE, FAKE, FAKE, 0.05, FAKE, None, 9, FAKE, big, None) == -1
    # workspace too small
    assert c(10, 10, FAKE, FAKE, FAKE, 0.05, FAKE, None, 0, FAKE, 1024, None) == -3
    s = L.sb2_sigma
    assert s(10, 0, FAKE, FAKE, FAKE, FAKE, FAKE, 0, FAKE, big, None) == -2
    assert s(10, 2, FAKE, None, FAKE, FAKE, FAKE, 0, FAKE, big, None) == -1
    assert s(10, 2, FAKE, FAKE, FAKE, FAKE, FAKE, 0, FAKE, 16, None) == -3
    r = L.sb2_rho_step
    assert r(0, FAKE, FAKE, FAKE, 0.05, FAKE, FAKE, big, None) == -2
    assert r(5, FAKE, FAKE, FAKE, 0.0, FAKE, FAKE, big, None) == -1
    assert r(5, FAKE, FAKE, FAKE, 0.05, FAKE, FAKE, 8, None) == -3


def test_backward_precision_and_batched_argument_errors(L):
    big = 1 << 40
    b = L.sb2_collision_backward
    assert b(10, 10, FAKE, FAKE, FAKE, 0.05, FAKE, FAKE, FAKE, FAKE, 1, FAKE, big, None) == -5
    assert b(0, 10, FAKE, FAKE, FAKE, 0.05, FAKE, FAKE, FAKE, FAKE, 0, FAKE, big, None) == -2
    assert L.sb2_collision_batched(0, None, 0, FAKE, big, None) in (-1, -2)
    desc = (_lib.SystemDesc * 1)()
    desc[0].N, desc[0].T, desc[0].dt = 10, 5, 0.05
    desc[0].v = desc[0].h = desc[0].rho_hist = desc[0].I_out = FAKE
    assert L.sb2_collision_batched(1, desc, 0, FAKE, 16, None) == -3
    desc[0].N = 0
    assert L.sb2_collision_batched(1, desc, 0, FAKE, big, None) == -2


def test_python_binding_rejects_cpu_tensors():
    import torch
    v = torch.zeros((2, 2, 2, 2), dtype=torch.float64)
    g = torch.zeros((1, 2, 2), dtype=torch.complex128)
    with pytest.raises(TypeError):
        _lib.sb2_sigma(v, g, g)
    assert ctypes.sizeof(_lib.SystemDesc) >= 48


def test_autotune_arguments_and_tuning_table(L):
    big = 1 << 40
    a = L.sb2_autotune
    assert a(0, 10, FAKE, FAKE, FAKE, 0.05, 0, FAKE, big, None, None, None, None) == -2
    assert a(10, 0, FAKE, FAKE, FAKE, 0.05, 0, FAKE, big, None, None, None, None) == -2
    assert a(10, 10, None, FAKE, FAKE, 0.05, 0, FAKE, big, None, None, None, None) == -1
    assert a(10, 10, FAKE, FAKE, FAKE, 0.0, 0, FAKE, big, None, None, None, None) == -1
    assert a(10, 10, FAKE, FAKE, FAKE, 0.05, 5, FAKE, big, None, None, None, None) == -1
    assert a(10, 10, FAKE, FAKE, FAKE, 0.05, 0, FAKE, 64, None, None, None, None) == -3
    ws = _lib.sb2_workspace_size
    assert ws("autotune", 10, 20, "fp16x3") > ws("collision", 10, 1, "fp16x3")
    s = L.sb2_set_tuning
    assert s(0, 0, 768, 100, 512) == -1
    assert s(10, 9, 768, 100, 512) == -1
    assert s(10, 0, 0, 100, 512) == -1
    assert s(10, 0, 768, 5, 512) == -1
    assert s(10, 0, 768, 201, 512) == -1
    assert s(10, 0, 768, 100, -1) == -1
    # workspace sizes do not depend on the tuned values
    before = [ws(op, 23, 7, p) for op in ("sigma", "collision") for p in ("fp64", "fp32", "fp16x3")]
    for p in (0, 1, 2):
        assert s(23, p, 1, 200, 0) == 0
    after = [ws(op, 23, 7, p) for op in ("sigma", "collision") for p in ("fp64", "fp32", "fp16x3")]
    for p in (0, 1, 2):
        assert s(23, p, 768, 100, 512) == 0      # back to the defaults
    assert before == after


def test_noalloc_entry_rejects_before_touching_the_device(L):
    c = L.sb2_collision_noalloc
    assert c(0, 10, FAKE, FAKE, FAKE, 0.05, FAKE, None, 0, None) == -2
    assert c(10, 10, None, FAKE, FAKE, 0.05, FAKE, None, 0, None) == -1
    assert c(10, 10, FAKE, FAKE, FAKE, -1.0, FAKE, None, 0, None) == -1
    # larger than the static scratch buffer (even one past time per pass)
    for n, prec in ((128, 2), (64, 1), (48, 0)):
        assert c(n, 100, FAKE, FAKE, FAKE, 0.05, FAKE, None, prec, None) == -6
    assert b"static buffer" in L.sb2_status_string(-6)


def test_split_bf16_is_recognised_but_not_built(L):
    big = 1 << 40
    bf16 = 3
    assert L.sb2_sigma(10, 2, FAKE, FAKE, FAKE, FAKE, FAKE, bf16, FAKE, big, None) == -5
    assert L.sb2_collision(10, 10, FAKE, FAKE, FAKE, 0.05, FAKE, None, bf16, FAKE, big, None) == -5
    assert L.sb2_collision_noalloc(10, 10, FAKE, FAKE, FAKE, 0.05, FAKE, None, bf16, None) == -5
    assert L.sb2_collision_prop(10, 10, FAKE, FAKE, FAKE, 0.05, FAKE, None, bf16, FAKE, big, None) == -5
    assert L.sb2_collision_backward(10, 10, FAKE, FAKE, FAKE, 0.05, FAKE, FAKE, FAKE, FAKE, bf16, FAKE, big,
                                    None) == -5
    assert L.sb2_gkba_propagate(10, 0, 1, FAKE, FAKE, FAKE, FAKE, None, 0.05, 3, bf16, FAKE, big, None) == -5
    assert L.sb2_autotune(10, 10, FAKE, FAKE, FAKE, 0.05, bf16, FAKE, big, None, None, None, None) == -5
    assert L.sb2_set_tuning(10, bf16, 768, 100, 512) == -5
    arr = (_lib.SystemDesc * 1)()
    arr[0].N, arr[0].T, arr[0].dt = 10, 10, 0.05
    arr[0].v = arr[0].h = arr[0].rho_hist = arr[0].I_out = FAKE
    assert L.sb2_collision_batched(1, arr, bf16, FAKE, big, None) == -5
    assert L.sb2_batched_workspace_size(1, arr, bf16) == 0
    for op in range(8):
        assert _lib.sb2_workspace_size(op, 10, 10, bf16) == 0
    # an unknown precision stays an invalid argument
    assert L.sb2_collision(10, 10, FAKE, FAKE, FAKE, 0.05, FAKE, None, 4, FAKE, big, None) == -1
    assert b"BF16" in L.sb2_status_string(-5)
    assert b"SB2_CHECK" in L.sb2_status_string(-7)
