"""The Python mirrors refuse buffers smaller than what the call accesses
(the C ABI takes bare pointers and cannot see sizes), before anything is
launched; buffers of the right size pass that check (and then fail here only
because CPU tensors are not device tensors)."""
import pytest
import torch

import paper_2602_20063_amd as shm


def f32(*shape):
    return torch.zeros(shape, dtype=torch.float32)


def expect(fn, *args, ok=False):
    with pytest.raises(ValueError) as e:
        fn(*args)
    assert ("device tensors" in str(e.value)) == ok, str(e.value)
    if not ok:
        assert "bytes" in str(e.value)


def test_query_mirror_sizes():
    N, n, q = 4, 3, 10
    lut = f32(n, 6, N + 2, N + 2, 4)
    args = [lut, shm.SHM_F32, shm.SHM_LAYOUT_TEXEL, N, n, f32(n * q, 3), q, f32(n * q, 4)]
    expect(shm.shm_query_value_grad, *args, ok=True)
    bad = list(args)
    bad[0] = f32(n - 1, 6, N + 2, N + 2, 4)
    expect(shm.shm_query_value_grad, *bad)
    bad = list(args)
    bad[5] = f32(n * q - 1, 3)
    expect(shm.shm_query_value_grad, *bad)
    bad = list(args)
    bad[7] = f32(n * q, 3)
    expect(shm.shm_query_value_grad, *bad)
    expect(shm.shm_query_value_grad, *args, f32(n * q - 1, 3))  # normal
    # the CELL layout needs 16 floats per cell
    cell = [f32(n, 6, N + 1, N + 1, 15), shm.SHM_F32, shm.SHM_LAYOUT_CELL] + args[3:]
    expect(shm.shm_query_value_grad, *cell)
    # FP16 data: half the bytes of FP32
    h = [torch.zeros((n, 6, N + 2, N + 2, 4), dtype=torch.float16), shm.SHM_F16] + args[2:]
    expect(shm.shm_query_value_grad, *h, ok=True)
    foot = [lut, shm.SHM_F32, shm.SHM_LAYOUT_TEXEL, N, n, f32(n * q, 3), q]
    expect(shm.shm_gather_footprints, *foot, f32(n * q, 16), ok=True)
    expect(shm.shm_gather_footprints, *foot, f32(n * q, 15))


def test_bake_and_backward_mirror_sizes():
    L, N, n = 3, 5, 2
    expect(shm.shm_bake_sh_lut_noalloc, f32(n, (L + 1) ** 2), L, N, n, shm.SHM_F32, f32(n, 6, N + 2, N + 2, 4), ok=True)
    expect(shm.shm_bake_sh_lut_noalloc, f32(n, (L + 1) ** 2 - 1), L, N, n, shm.SHM_F32, f32(n, 6, N + 2, N + 2, 4))
    expect(shm.shm_bake_sh_lut_noalloc, f32(n, (L + 1) ** 2), L, N, n, shm.SHM_F32, f32(n, 6, N + 2, N + 2, 3))
    Q = 7
    lut = f32(1, 6, N + 2, N + 2, 4)
    ws = torch.zeros(shm.shm_backward_workspace(N, 1, Q), dtype=torch.uint8)
    args = [lut, N, 1, f32(Q, 3), Q, f32(Q, 4), f32(1, 6, N + 2, N + 2, 4), f32(Q, 3), ws, 0]
    expect(shm.shm_query_backward, *args, ok=True)
    bad = list(args)
    bad[6] = f32(1, 6, N + 2, N + 1, 4)
    expect(shm.shm_query_backward, *bad)
    bad = list(args)
    bad[5] = f32(Q - 1, 4)
    expect(shm.shm_query_backward, *bad)


def test_trace_and_probe_mirror_sizes():
    N, P = 6, 9
    lut = f32(6, N + 2, N + 2, 4)
    rays = [f32(P, 3), f32(P, 3), P, 20, 8, 3, f32(P), f32(P, 4)]
    expect(shm.shm_trace_radial, lut, shm.SHM_F32, N, (0, 0, 0), 1.5, *rays, ok=True)
    expect(shm.shm_trace_radial, lut, shm.SHM_F32, N, (0, 0, 0), 1.5, *rays[:-1], f32(P - 1, 4))
    expect(shm.shm_trace_radial, f32(6, N + 2, N + 2, 3), shm.SHM_F32, N, (0, 0, 0), 1.5, *rays)
    prm = shm.shm_trace_params(1.0, 0, 20, 8, 3, 0.0, 0.0, 0, 0, None)
    u8 = torch.zeros(P, dtype=torch.uint8)
    ex = [lut, shm.SHM_F32, N, (0, 0, 0), 1.5, prm, f32(P, 3), f32(P, 3), P, f32(P), f32(P, 4), f32(P, 3)]
    expect(shm.shm_trace_radial_ex, *ex, torch.zeros(P, dtype=torch.int8), u8, ok=True)  # sign int8, evals uint8
    expect(shm.shm_trace_radial_ex, *ex, torch.zeros(P, dtype=torch.int8), u8[:-1])
    prm.flags = shm.SHM_CELL_LUT  # a CELL LUT of the same N is larger than the TEXEL one
    expect(shm.shm_trace_radial_ex, *ex, None, None)
    base = f32(4 * 1024)
    expect(shm.shm_probe_gather, base, 4096, 4, 10, 64, 1, shm.SHM_PROBE_OUT, None, f32(40, 4), ok=True)
    expect(shm.shm_probe_gather, base, 4096, 5, 10, 64, 1, shm.SHM_PROBE_OUT, None, f32(50, 4))
    expect(shm.shm_probe_gather, base, 4096, 4, 10, 64, 1, shm.SHM_PROBE_OUT | shm.SHM_PROBE_DIRS, f32(39, 3),
           f32(40, 4))
