"""Ray casting on the GPU against the FP64 oracle's schedule on the same
LUT data."""
import numpy as np
import pytest
import torch

import oracle
import paper_2602_20063_amd as shm
import workloads
from parity import angle_deg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def gpu(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def trace_both(lut32, rmax, o, d, dtype=torch.float32):
    t, out, n = shm.trace(gpu(lut32, dtype), (0.0, 0.0, 0.0), rmax, gpu(o), gpu(d))
    torch.cuda.synchronize()
    ref = oracle.trace(lut32.astype(np.float64) if dtype == torch.float32 else lut32.astype(np.float16).astype(np.float64),
                       np.zeros(3), rmax, o, d)
    return (t.cpu().numpy(), out.cpu().numpy(), n.cpu().numpy()), ref


def compare(g, ref, what, max_disagree=0.002):
    tg, og, ng = g
    tr, orf, nr = ref
    hg, hr = np.isfinite(tg), np.isfinite(tr)
    disagree = np.mean(hg != hr)
    assert disagree <= max_disagree, f"{what}: hit mask disagreement {disagree:.4f}"
    both = hg & hr
    rel = np.abs(tg[both] - tr[both]) / tr[both]
    assert np.median(rel) < 1e-6, f"{what}: median |dt|/t {np.median(rel):.2e}"
    assert np.mean(rel < 1e-4) > 0.995, f"{what}: |dt|/t tail"
    ang = angle_deg(ng[both], nr[both])
    assert np.median(ang) < 1e-3 and np.mean(ang < 0.05) > 0.995, f"{what}: normal angle"
    assert np.isnan(og[~hg]).all() and np.isinf(tg[~hg]).all()


def test_trace_sh_glyph():
    c = workloads.sh_glyph_coeffs(8, 1, np.random.default_rng(3))[0]
    N = 32
    lut = oracle.bake_sh(c, N).astype(np.float32)
    rmax = oracle.rmax_bound(lut.astype(np.float64)) * 1.0001
    o, d = workloads.camera_rays(160, 120)
    g, ref = trace_both(lut, rmax, o, d)
    compare(g, ref, "glyph")


def test_trace_bumps_fd_lut():
    """Workload 3 surface (64 bumps) at reduced resolution, FP32 and FP16."""
    mu, amp, width = workloads.bump_params(workloads.rng_for(3))
    N = 64
    dirs = oracle.margin_dirs(N)
    samples = workloads.bumps_value(mu, amp, width, 1.0, dirs.reshape(-1, 3)).reshape(6, N + 4, N + 4)
    lut = oracle.bake_fd(samples, N).astype(np.float32)
    rmax = oracle.rmax_bound(lut.astype(np.float64)) * 1.0001
    o, d = workloads.camera_rays(192, 108)
    g, ref = trace_both(lut, rmax, o, d)
    compare(g, ref, "bumps fp32")
    g16, ref16 = trace_both(lut, rmax, o, d, dtype=torch.float16)
    compare(g16, ref16, "bumps fp16")


def test_trace_constant_sphere_and_misses():
    N = 8
    lut = np.zeros((6, N + 2, N + 2, 4), np.float32)
    lut[..., 0] = 0.75
    o, d = workloads.camera_rays(64, 64, eye=(0.0, 0.0, 2.0), vfov_deg=60.0)
    g, ref = trace_both(lut, 0.8, o, d)
    compare(g, ref, "sphere", max_disagree=0.0)
    tg = g[0]
    hit = np.isfinite(tg)
    oo = o.astype(np.float64)
    dd = d.astype(np.float64) / np.linalg.norm(d.astype(np.float64), axis=1, keepdims=True)
    b = np.sum(oo * dd, axis=1)
    disc = b * b - (np.sum(oo * oo, axis=1) - 0.75 ** 2)
    assert np.array_equal(hit, disc > 0) or np.mean(hit != (disc > 0)) < 0.002
    te = -b[hit] - np.sqrt(disc[hit])
    assert np.abs(tg[hit] - te).max() < 1e-5


@pytest.mark.parametrize("W,H", [(67, 29), (8, 8), (1, 5), (200, 1)])
def test_trace_image_tiles_same_bits(W, H):
    """Rays of a row-major image traced one wavefront per 8 x 8 tile (ragged
    right and bottom edges) give the same bits as one lane per ray in ray
    order, for every output and both LUT precisions, fixed and adaptive
    budgets; and match the oracle."""
    mu, amp, width = workloads.bump_params(workloads.rng_for(3))
    N = 64
    dirs = oracle.margin_dirs(N)
    samples = workloads.bumps_value(mu, amp, width, 1.0, dirs.reshape(-1, 3)).reshape(6, N + 4, N + 4)
    lut = oracle.bake_fd(samples, N).astype(np.float32)
    rmax = oracle.rmax_bound(lut.astype(np.float64)) * 1.0001
    o, d = workloads.camera_rays(W, H, vfov_deg=25.0)
    og, dg = gpu(o), gpu(d)
    for dt in (torch.float32, torch.float16):
        lt = gpu(lut, dt)
        lin = shm.trace(lt, (0.0, 0.0, 0.0), rmax, og, dg)
        til = shm.trace(lt, (0.0, 0.0, 0.0), rmax, og, dg, image_width=W)
        for a, b in zip(lin, til):
            assert same_bits(a, b)
        lin = shm.trace_ex(lt, (0.0, 0.0, 0.0), rmax, og, dg, px_per_unit=300.0, eps_px=0.125, n_bisect=12)
        til = shm.trace_ex(lt, (0.0, 0.0, 0.0), rmax, og, dg, px_per_unit=300.0, eps_px=0.125, n_bisect=12,
                           image_width=W)
        for a, b in zip(lin, til):
            assert same_bits(a, b)
    g = tuple(x.cpu().numpy() for x in shm.trace(gpu(lut), (0.0, 0.0, 0.0), rmax, og, dg, image_width=W))
    torch.cuda.synchronize()
    ref = oracle.trace(lut.astype(np.float64), np.zeros(3), rmax, o, d)
    assert np.isfinite(ref[0]).any()
    compare(g, ref, f"tiled {W}x{H}", max_disagree=max(0.002, 1.5 / (W * H)))


def same_bits(a, b):
    if a.dtype == torch.float32:
        return torch.equal(a.view(torch.int32), b.view(torch.int32))
    return torch.equal(a, b)


def bumps_lut(N):
    mu, amp, width = workloads.bump_params(workloads.rng_for(3))
    md = oracle.margin_dirs(N)
    samples = workloads.bumps_value(mu, amp, width, 1.0, md.reshape(-1, 3)).reshape(6, N + 4, N + 4)
    return oracle.bake_fd(samples, N).astype(np.float32)


@pytest.mark.parametrize("B", [1, 5, 8, 64])
def test_bound_map_bounds_the_reconstruction(B):
    """Every block's bound is the oracle's largest control point over the
    (widened) cells of the block, and no query of a direction in the block
    exceeds it."""
    N = 40
    lut = bumps_lut(N)
    bmap = shm.lut_bound_map(gpu(lut), blocks=B).cpu().numpy()
    lut64 = lut.astype(np.float64)
    rng = np.random.default_rng(B)
    for f, bj, bi in [(0, 0, 0), (3, B - 1, B - 1), (5, B // 2, (B - 1) // 3)] + [tuple(x) for x in rng.integers(0, [6, B, B], (6, 3))]:
        lo = lambda b: max((2 * b * N + B) // (2 * B) - 1, 0)
        hi = lambda b: min((2 * (b + 1) * N + B) // (2 * B) + 1, N)
        want = max(0.0, max(oracle.cell_bezier(lut64, f, i0, j0).max()
                            for j0 in range(lo(bj), hi(bj) + 1) for i0 in range(lo(bi), hi(bi) + 1)))
        assert abs(bmap[f, bj, bi] - want) <= 1e-6 * want, (f, bj, bi, bmap[f, bj, bi], want)
    dirs = workloads.uniform_dirs(200000, rng)
    r = shm.query(gpu(lut)[None], gpu(dirs)).cpu().numpy()[:, 0]
    face, i0, j0, s, t = oracle.locate(dirs, N)
    bu = np.clip(np.floor((i0 + s - 0.5) / N * B).astype(int), 0, B - 1)
    bv = np.clip(np.floor((j0 + t - 0.5) / N * B).astype(int), 0, B - 1)
    assert (r <= bmap[face, bv, bu] * (1 + 1e-6)).all()


@pytest.mark.parametrize("dt", [torch.float32, torch.float16])
def test_trace_bound_map_same_bits(dt):
    """Skipping the march samples the bound map proves outside the surface
    changes no output bit and only lowers the evaluation counts; fixed and
    adaptive budgets, plain and signed radius, image tiles and ray order."""
    N = 64
    lut = gpu(bumps_lut(N), dt)
    rmax = float(shm.lut_rmax(lut).item()) * 1.0001
    o, d = workloads.camera_rays(67, 29, vfov_deg=30.0)
    og, dg = gpu(o), gpu(d)
    for signed, px in ((False, 0.0), (True, 300.0)):
        bmap = shm.lut_bound_map(lut, blocks=16, signed=signed)
        for w in (0, 67):
            kw = dict(signed=signed, px_per_unit=px, eps_px=0.125, n_bisect=12, image_width=w)
            a = shm.trace_ex(lut, (0.0, 0.0, 0.0), rmax, og, dg, **kw)
            b = shm.trace_ex(lut, (0.0, 0.0, 0.0), rmax, og, dg, bound_map=bmap, **kw)
            for x, y in zip(a[:4], b[:4]):
                assert same_bits(x, y)
            ea, eb = a[4].int(), b[4].int()
            assert (eb <= ea).all() and eb.sum() < ea.sum()
    a = shm.trace(lut, (0.0, 0.0, 0.0), rmax, og, dg)
    b = shm.trace(lut, (0.0, 0.0, 0.0), rmax, og, dg, bound_map=shm.lut_bound_map(lut, blocks=8))
    for x, y in zip(a, b):
        assert same_bits(x, y)


def test_trace_cells_same_bits_and_f16_accuracy():
    """Ray casting a CELL LUT: FP32 cells give the bits of the FP32 texel
    LUT (the same footprints), bounds and bound maps included; FP16 cells
    (value differences, from the FP32 data) give the bits of the FP32 cells
    they decode to, with and without the bound map; and their normals stay
    far closer to the FP32 trace's than plain FP16 texels'."""
    from parity import decode_f16_cells
    N = 64
    lut = gpu(bumps_lut(N))[None]
    cells = shm.to_cells(lut)
    c16 = shm.cells_to_f16(cells)
    dec = gpu(decode_f16_cells(c16.cpu().numpy()))
    o, d = workloads.camera_rays(96, 64, vfov_deg=30.0)
    og, dg = gpu(o), gpu(d)
    rmax = float(shm.lut_rmax(lut[0]).item()) * 1.0001
    assert same_bits(shm.lut_rmax(cells[0]), shm.lut_rmax(lut[0]))
    assert same_bits(shm.lut_bound_map(cells[0], blocks=16), shm.lut_bound_map(lut[0], blocks=16))
    assert same_bits(shm.lut_bound_map(c16[0], blocks=16), shm.lut_bound_map(dec[0], blocks=16))
    assert same_bits(shm.lut_rmax(c16[0]), shm.lut_rmax(dec[0]))
    t32 = shm.trace(lut[0], (0.0, 0.0, 0.0), rmax, og, dg)
    for x, y in zip(t32, shm.trace(cells[0], (0.0, 0.0, 0.0), rmax, og, dg)):
        assert same_bits(x, y)
    rmax16 = float(shm.lut_rmax(c16[0]).item()) * 1.0001
    kw = dict(image_width=96, bound_map=shm.lut_bound_map(c16[0]))
    a = shm.trace(c16[0], (0.0, 0.0, 0.0), rmax16, og, dg)
    for x, y in zip(a, shm.trace(dec[0], (0.0, 0.0, 0.0), rmax16, og, dg)):
        assert same_bits(x, y)
    for x, y in zip(a, shm.trace(c16[0], (0.0, 0.0, 0.0), rmax16, og, dg, **kw)):
        assert same_bits(x, y)
    t16 = shm.trace(lut[0].half(), (0.0, 0.0, 0.0), rmax16, og, dg)
    hit = torch.isfinite(t32[0]) & torch.isfinite(a[0]) & torch.isfinite(t16[0])
    assert hit.float().mean().item() > 0.2
    ang_c = angle_deg(a[2][hit].cpu().numpy(), t32[2][hit].cpu().numpy())
    ang_t = angle_deg(t16[2][hit].cpu().numpy(), t32[2][hit].cpu().numpy())
    print(f"FP16 trace normal vs FP32, mean / max deg: cells {ang_c.mean():.3g} / {ang_c.max():.3g}, "
          f"texels {ang_t.mean():.3g} / {ang_t.max():.3g}")
    print(f"  median {np.median(ang_c):.3g} / {np.median(ang_t):.3g}, p99 {np.quantile(ang_c, 0.99):.3g} / "
          f"{np.quantile(ang_t, 0.99):.3g}")
    # (a few grazing rays, where a small shift of the hit swings the normal,
    # make up the tails of both)
    assert ang_c.mean() < 0.05 * ang_t.mean() and np.median(ang_c) < 0.05 * np.median(ang_t)
