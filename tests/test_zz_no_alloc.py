"""The SH bake without a workspace (shm_bake_sh_lut_noalloc) against the bake
with a caller workspace (shm_bake_sh_lut): the same kernels on the same
inputs, so the LUTs must be bit for bit equal, on two calls in a row, the
second smaller than the first (the scratch array keeps the first call's
table; the second must not read any of it)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2602_20063_amd as shm
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def bake_both(c32, L, N, dtype):
    c_t = torch.as_tensor(c32).to(DEV)
    n = c32.shape[0]
    ref = shm.bake_sh(c_t, N, dtype=dtype)  # the workspace entry point
    out = torch.full_like(ref, float("nan"))
    code = shm.SHM_F16 if dtype == torch.float16 else shm.SHM_F32
    shm.shm_bake_sh_lut_noalloc(c_t, L, N, n, code, out)
    torch.cuda.synchronize()
    return ref, out


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_noalloc_bake_matches_workspace_bake_twice(dtype):
    rng = np.random.default_rng(71)
    calls = [(8, 32, 300), (4, 10, 3)]  # the second call is smaller
    for L, N, n in calls:
        c32 = workloads.sh_glyph_coeffs(L, n, rng).astype(np.float32)
        ref, out = bake_both(c32, L, N, dtype)
        view = torch.int16 if dtype == torch.float16 else torch.int32
        assert torch.equal(out.view(view), ref.view(view)), (L, N, n)


def test_noalloc_bake_largest_table_and_limit():
    """The largest SH order fits at N = 32 (and goes through the LDS-staged
    contraction); a table beyond the scratch size is refused with a message
    naming the sizes, before anything is enqueued."""
    rng = np.random.default_rng(72)
    assert shm.shm_bake_sh_lut_workspace(16, 32) <= shm.SHM_BAKE_NOALLOC_MAX_BYTES
    c32 = workloads.sh_glyph_coeffs(16, 5, rng).astype(np.float32)
    ref, out = bake_both(c32, 16, 32, torch.float32)
    assert torch.equal(out.view(torch.int32), ref.view(torch.int32))
    assert shm.shm_bake_sh_lut_workspace(16, 64) > shm.SHM_BAKE_NOALLOC_MAX_BYTES
    c_t = torch.zeros((1, 289), device=DEV)
    lut = torch.empty((1, 6, 66, 66, 4), device=DEV)
    rc = shm.lib().shm_bake_sh_lut_noalloc(ctypes.c_void_p(c_t.data_ptr()), 16, 64, 1, shm.SHM_F32,
                                           ctypes.c_void_p(lut.data_ptr()), None)
    assert rc == shm.SHM_ERR_UNSUPPORTED
    assert "scratch" in shm.shm_last_error()
