"""GPU bake (SH basis + MFMA contraction; finite-difference mode; bound)
against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2602_20063_amd as shm
import workloads
from parity import check_value_grad

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rng(k):
    return np.random.default_rng(4242 + k)


def gpu(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def check_lut(g, ref, what, val_rtol=1e-5, der_rtol=1e-4):
    """R channel <= val_rtol relative; derivative channels <= der_rtol of
    that channel's RMS."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    dv = np.abs(g[..., 0] - ref[..., 0]) / np.abs(ref[..., 0]).clip(1e-30)
    assert dv.max() <= val_rtol, f"{what}: R channel {dv.max():.3e}"
    for ch in (1, 2, 3):
        rms = np.sqrt(np.mean(ref[..., ch] ** 2))
        if rms == 0.0:  # constant function: derivative channels vanish
            assert np.abs(g[..., ch]).max() <= 1e-6, f"{what}: channel {ch} not zero"
            continue
        e = np.abs(g[..., ch] - ref[..., ch]).max() / rms
        assert e <= der_rtol, f"{what}: channel {ch} error {e:.3e} of RMS"


# every register-resident contraction width (L = 0 .. 8: 1, 1, 2, 4, 6, 9, 12,
# 16, 20 K steps of 4) and the LDS-staged kernel above it (L >= 9)
@pytest.mark.parametrize("L,N,n", [(4, 10, 1), (8, 32, 70), (2, 5, 3), (0, 3, 2), (12, 16, 5), (16, 8, 4), (1, 7, 2),
                                   (3, 9, 3), (5, 11, 2), (6, 12, 2), (7, 13, 2), (9, 8, 2)])
def test_bake_sh_matches_oracle(L, N, n):
    c = workloads.sh_glyph_coeffs(L, n, rng(L * 100 + N))
    c32 = c.astype(np.float32)
    lut = shm.bake_sh(gpu(c32), N)
    torch.cuda.synchronize()
    ref = oracle.bake_sh(c32.astype(np.float64), N)
    check_lut(lut.cpu().numpy().reshape(ref.shape), ref, f"L={L} N={N}")


def test_bake_fp16_output():
    L, N, n = 8, 32, 9
    c32 = workloads.sh_glyph_coeffs(L, n, rng(1)).astype(np.float32)
    l16 = shm.bake_sh(gpu(c32), N, dtype=torch.float16)
    l32 = shm.bake_sh(gpu(c32), N)
    torch.cuda.synchronize()
    assert torch.equal(l16, l32.half())


def test_bake_then_query_end_to_end():
    """GPU bake -> GPU query vs oracle bake -> oracle query (both from the
    same FP32 coefficients), 256 glyphs of the glyph field: value within
    1e-5 and gradient within 1e-4 (relative to max(|grad|, RMS |grad|)) of
    FP64 end to end.  The gradient of the reconstruction differences
    neighbouring texels' values, so this holds only if the bake's value
    channel carries little more than its FP32 storage rounding."""
    L, N, n = 8, 32, 256
    c32 = workloads.sh_glyph_coeffs(L, n, workloads.rng_for(2)).astype(np.float32)
    dirs = workloads.uniform_dirs(n * 256, workloads.rng_for(2))
    lut = shm.bake_sh(gpu(c32), N)
    out = shm.query(shm.to_cells(lut), gpu(dirs), q_per_obj=256, layout=shm.SHM_LAYOUT_CELL).cpu().numpy()
    ref_lut = oracle.bake_sh(c32.astype(np.float64), N)
    off = np.arange(n) * (ref_lut[0].size // 4)
    ref = oracle.query_objects(ref_lut.reshape(-1), off, [N] * n, np.arange(n) * 256, [256] * n, dirs)
    st = check_value_grad(out, ref, "bake + query end to end")
    print("end to end vs FP64:", st)


@pytest.mark.parametrize("L,N", [(0, 4), (1, 6), (12, 16)])
def test_l0_term_added_once(L, N):
    """The l = 0 term leaves the contraction and enters the value channel
    once: a constant function (only c_00) bakes to c_00 Y_00 rounded once,
    with exactly zero derivative channels, through both contraction kernels
    (register-resident for L <= 8, LDS-staged above)."""
    n = 3
    c = np.zeros((n, (L + 1) ** 2), np.float32)
    c[:, 0] = np.array([3.5449077, -1.25, 7.0], np.float32)
    lut = shm.bake_sh(gpu(c), N).cpu().numpy().reshape(n, -1, 4)
    for o in range(n):
        expect = np.float32(np.float64(c[o, 0]) * 0.28209479177387814347)
        assert np.all(lut[o, :, 0] == expect)
        assert np.all(lut[o, :, 1:] == 0.0)


def test_margin_dirs_and_fd_bake():
    N = 24
    d = shm.margin_dirs(N, DEV).cpu().numpy()
    ref_d = oracle.margin_dirs(N)
    assert np.abs(d - ref_d).max() < 4e-7
    mu, amp, width = workloads.bump_params(rng(2), 16)
    samples = workloads.bumps_value(mu, amp, width, 1.0, d.reshape(-1, 3)).reshape(6, N + 4, N + 4)
    lut = shm.bake_fd(gpu(samples.astype(np.float32)), N)
    ref = oracle.bake_fd(samples.astype(np.float32).astype(np.float64), N)
    check_lut(lut.cpu().numpy()[0], ref, "fd bake", val_rtol=0, der_rtol=1e-6)
    l16 = shm.bake_fd(gpu(samples.astype(np.float32)), N, dtype=torch.float16)
    assert torch.equal(l16, lut.half())


def test_lut_rmax_bound():
    for k, N in enumerate((6, 33, 128)):
        c = workloads.sh_glyph_coeffs(8, 1, rng(10 + k))[0]
        lut = oracle.bake_sh(c, N).astype(np.float32)
        g = shm.lut_rmax(gpu(lut)).item()
        ref = oracle.rmax_bound(lut.astype(np.float64))
        assert abs(g - ref) <= 2e-6 * ref, (N, g, ref)


@pytest.mark.parametrize("naive", [False, True])
def test_mip_level_matches_oracle(naive):
    """Mip chain (Sec. 4.7): three levels of a glyph map, GPU vs oracle on the
    same FP32 input level each time."""
    c = workloads.sh_glyph_coeffs(8, 1, rng(30))[0]
    lut = oracle.bake_sh(c, 32).astype(np.float32)
    for _ in range(3):
        g = shm.mip_level(gpu(lut), naive=naive).cpu().numpy()
        ref = oracle.mip_level(lut.astype(np.float64), naive=naive)
        check_lut(g, ref, f"mip naive={naive}", val_rtol=2e-6, der_rtol=2e-4)
        lut = g
