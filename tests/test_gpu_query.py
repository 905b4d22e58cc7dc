"""GPU parity of the query (value + spherical gradient) against the FP64
oracle, element by element on the same seeded inputs and the same LUT data.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2602_20063_amd as shm
import workloads
from parity import check_value_grad, angle_deg, decode_f16_cells
from oracle import ties

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def rng(k):
    return np.random.default_rng(777 + k)


def gpu(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def gpu_query(lut32, dirs, layout=shm.SHM_LAYOUT_TEXEL, dtype=torch.float32, q_per_obj=None, normals=False):
    lut_t = gpu(lut32, dtype)
    if layout == shm.SHM_LAYOUT_CELL:
        lut_t = shm.to_cells(lut_t.reshape((-1,) + lut_t.shape[-4:]))
    res = shm.query(lut_t, gpu(dirs), q_per_obj=q_per_obj, layout=layout, normals=normals)
    torch.cuda.synchronize()
    if normals:
        return res[0].cpu().numpy(), res[1].cpu().numpy()
    return res.cpu().numpy()


def edge_dirs():
    """Axis directions, face ties, sign ties, -0, cube corners, directions
    landing exactly on cell boundaries, subnormal to huge magnitudes and
    invalid directions."""
    d = [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
         [1, 1, 0], [1, -1, 0], [-1, 1, 1], [1, 1, 1], [-1, -1, -1], [0, 1, 1], [0, -1, -1],
         [-0.0, 0.0, 1.0], [1, -0.0, -0.0], [0.5, 0.5, 0.5], [3, 1, 2], [1e-30, 0, 0],
         [1e30, 1e29, -1e29],
         # subnormal, tiny and huge magnitudes: valid, the same directions
         [1e-42, 3e-43, -5e-43], [2e-39, -1e-39, 0], [1e-20, -1e-20, 5e-21], [3e38, -1e38, 2e38],
         [0, 0, 0], [np.nan, 1, 0], [np.inf, 0, 0]]
    return np.array(d, np.float32)


@pytest.mark.parametrize("layout", [shm.SHM_LAYOUT_TEXEL, shm.SHM_LAYOUT_CELL])
def test_query_cfg1_random_lut(layout):
    """Workload 1 shape (N=10, 65,536 directions) on arbitrary texel data."""
    r = rng(1)
    N = 10
    lut = workloads.random_lut(N, r)
    dirs = workloads.uniform_dirs(65536, workloads.rng_for(1))
    out = gpu_query(lut, dirs, layout)
    ref = oracle.query(lut, dirs)
    check_value_grad(out, ref, "cfg1 random lut")


def test_query_cfg1_sh_glyph_with_normals():
    c = workloads.sh_glyph_coeffs(4, 1, workloads.rng_for(1))[0]
    N = 10
    lut = oracle.bake_sh(c, N).astype(np.float32)
    dirs = workloads.uniform_dirs(65536, workloads.rng_for(1))
    out, nrm = gpu_query(lut, dirs, normals=True)
    ref, rn = oracle.query(lut, dirs, normals=True)
    check_value_grad(out, ref, "cfg1 glyph")
    assert angle_deg(nrm, rn).max() < 1e-3


def test_cell_keys_match_fp64_except_ties():
    """Faces identical to the oracle's; cells identical to the oracle's FP64
    decision except at ties (FP64 coordinate within the FP32 decision's
    rounding band of a cell edge), which are counted, printed and bounded."""
    dirs = np.concatenate([workloads.uniform_dirs(200000, rng(2)), edge_dirs()])
    total = 0
    for N in (1, 10, 32, 257, 1024):
        keys = shm.cell_keys(N, gpu(dirs)).cpu().numpy()
        r = ties.classify(keys, dirs, N)
        print(f"N={N}: {r['mismatches']} FP32/FP64 cell ties of {r['queries']} queries "
              f"({r['ties_in_band']} coordinates in the tie band)")
        assert r["ok"], (N, r)
        assert r["mismatches"] <= r["ties_in_band"]
        # the band is a few FP32 ulps of f wide, ~N ulp(1) at the face edges
        # (plus the hand-made edge directions, several of them exactly on
        # cell edges)
        assert r["ties_in_band"] <= 1e-6 * N * r["queries"] + len(edge_dirs()) + 10, (N, r)
        total += r["mismatches"]
    # workload 1 at full size
    dirs1 = workloads.uniform_dirs(65536, workloads.rng_for(1))
    r1 = ties.classify(shm.cell_keys(10, gpu(dirs1)).cpu().numpy(), dirs1, 10)
    print(f"workload 1 (N=10, 65,536 queries): {r1['mismatches']} ties ({r1['ties_in_band']} in band)")
    assert r1["ok"], r1


def test_cell_ties_exact_edges():
    """Directions whose FP64 coordinate sits exactly on a cell edge (f an
    integer, representable in both precisions) decide identically: the tie
    rule only admits mismatches where rounding can move f across the edge."""
    out = []
    for N in (2, 4, 8, 16, 32):
        for k in range(1, N + 1):
            u = (k - 0.5) / N  # f = k exactly
            for v in (0.3, 0.5, 0.77):
                out.append([1.0, -(2 * v - 1), -(2 * u - 1)])  # +X face: sc = -z, tc = -y
        dirs = np.array(out, np.float32)
        keys = shm.cell_keys(N, gpu(dirs)).cpu().numpy()
        r = ties.classify(keys, dirs, N)
        assert r["ok"] and r["mismatches"] == 0, (N, r)
        out = []


def test_layouts_agree_bitwise():
    r = rng(3)
    N = 17
    lut = workloads.random_lut(N, r, n_obj=3)
    dirs = workloads.uniform_dirs(3 * 1000, r)
    a = gpu_query(lut, dirs, shm.SHM_LAYOUT_TEXEL)
    b = gpu_query(lut, dirs, shm.SHM_LAYOUT_CELL)
    assert np.array_equal(a, b)


def test_edge_cases():
    r = rng(4)
    N = 8
    lut = workloads.random_lut(N, r)
    d = edge_dirs()
    out = gpu_query(lut, d)
    ref = oracle.query(lut, d)
    check_value_grad(out, ref, "edge dirs")
    assert np.isnan(out[-3:]).all()
    # texel-centre directions and exact cell-boundary directions
    N = 6
    lut = workloads.random_lut(N, r)
    dd = []
    for p in range(N + 1):
        u = p / N  # f = uN + 1/2 = p + 1/2 ... cell edges sit at u = (k - 1/2)/N
        for q in range(N + 1):
            v = (q + 0.5) / N
            for uu, vv in ((u, v), (np.clip((p - 0.5) / N, 0, 1), v)):
                dd.append([1.0, -(2 * vv - 1), -(2 * uu - 1)])  # +X face: sc = -z, tc = -y
    dd = np.array(dd, np.float32)
    check_value_grad(gpu_query(lut, dd), oracle.query(lut, dd), "boundaries")


def test_empty_and_ragged():
    r = rng(5)
    N = 12
    lut = workloads.random_lut(N, r, n_obj=4)
    for qpo in (1, 255, 257, 1000):
        dirs = workloads.uniform_dirs(4 * qpo, r)
        check_value_grad(gpu_query(lut, dirs, q_per_obj=qpo), oracle.query_objects(
            lut.reshape(-1), np.arange(4) * (lut.size // 16), [N] * 4, np.arange(4) * qpo, [qpo] * 4, dirs), f"qpo {qpo}")
    lut_t = gpu(lut)
    empty = torch.empty((0, 3), device=DEV)
    out = torch.empty((0, 4), device=DEV)
    shm.shm_query_value_grad(lut_t, shm.SHM_F32, 0, N, 4, empty, 0, out)


@pytest.mark.parametrize("N", [1, 2, 64, 512, 1024])
def test_resolution_extremes(N):
    r = rng(6 + N)
    lut = workloads.random_lut(N, r)
    dirs = workloads.uniform_dirs(20000, r)
    check_value_grad(gpu_query(lut, dirs), oracle.query(lut, dirs), f"N={N}")


def test_large_n_smooth_lut_gradient_accuracy():
    """Smooth data at N=512: gradient relative accuracy must hold even where
    r_u is O(1) while texel differences are O(1/N)."""
    c = workloads.sh_glyph_coeffs(8, 1, rng(7))[0]
    N = 512
    lut = oracle.bake_sh(c, N).astype(np.float32)
    dirs = workloads.uniform_dirs(50000, rng(8))
    check_value_grad(gpu_query(lut, dirs), oracle.query(lut, dirs), "N=512 glyph")


def test_fp16_lut():
    """FP16 storage: FP32 arithmetic on the decoded values matches the oracle
    on the same (FP16-rounded) data; the error against the FP32 LUT is the
    quantisation error and is only bounded loosely here (it grows ~ N)."""
    c = workloads.sh_glyph_coeffs(8, 1, rng(9))[0]
    N = 32
    lut = oracle.bake_sh(c, N)
    lut16 = lut.astype(np.float16)
    dirs = workloads.uniform_dirs(65536, rng(10))
    for layout in (shm.SHM_LAYOUT_TEXEL, shm.SHM_LAYOUT_CELL):
        out = gpu_query(lut16.astype(np.float32), dirs, layout, dtype=torch.float16)
        check_value_grad(out, oracle.query(lut16.astype(np.float64), dirs), "fp16 same data")
    ref64 = oracle.query(lut, dirs)
    assert np.abs(out[:, 0] - ref64[:, 0]).max() < 2e-3


def test_cfg2_shape_reduced_and_sampled_full():
    """Workload 2 layout (glyph-contiguous queries, 256 per glyph, N=32,
    L=8): 256 glyphs element by element."""
    n = 256
    c = workloads.sh_glyph_coeffs(8, n, workloads.rng_for(2))
    lut = oracle.bake_sh(c, 32).astype(np.float32)
    dirs = workloads.uniform_dirs(n * 256, workloads.rng_for(2))
    out = gpu_query(lut, dirs, q_per_obj=256)
    ref = oracle.query_objects(lut.reshape(-1), np.arange(n) * (lut[0].size // 4), [32] * n, np.arange(n) * 256,
                               [256] * n, dirs)
    check_value_grad(out, ref, "cfg2 reduced")


def test_count_invalid_matches_the_nan_rows():
    """The bad-query counter counts exactly the directions the query answers
    with NaN: zero vectors (+-0), NaN or Inf components; tiny, huge and
    subnormal nonzero vectors are valid.  Counts add up across calls."""
    rng = np.random.default_rng(13)
    Q = 100003
    d = workloads.uniform_dirs(Q, rng) * rng.uniform(1e-3, 1e3, (Q, 1)).astype(np.float32)
    k = rng.choice(Q, 600, replace=False)
    d[k[:100]] = 0.0
    d[k[100:150]] = -0.0
    d[k[150:250], rng.integers(0, 3, 100)] = np.nan
    d[k[250:350], rng.integers(0, 3, 100)] = np.inf
    d[k[350:400], rng.integers(0, 3, 50)] = -np.inf
    d[k[400:450]] = np.float32(1e-42)           # subnormal, valid
    d[k[450:500]] = np.float32(3e38)            # huge, valid
    d[k[500:600]] = d[k[500:600]] * np.float32(1e-30)
    ref = int((~(np.isfinite(d).all(axis=1) & (np.abs(d).max(axis=1) > 0))).sum())
    assert ref == 400  # 150 zero vectors, 100 NaN, 150 Inf
    dirs = torch.as_tensor(d).to(DEV)
    assert shm.count_invalid(dirs) == ref
    c = torch.zeros(1, dtype=torch.int64, device=DEV)
    shm.shm_count_invalid(dirs, Q, c)
    shm.shm_count_invalid(dirs[:1000].contiguous(), 1000, c)
    lut = torch.as_tensor(workloads.random_lut(8, rng)).to(DEV)[None].contiguous()
    out = torch.empty((Q, 4), device=DEV)
    nrm = torch.empty((Q, 3), device=DEV)
    shm.shm_query_value_grad(lut, shm.SHM_F32, shm.SHM_LAYOUT_TEXEL, 8, 1, dirs, Q, out, nrm)
    nan_rows = torch.isnan(out).all(dim=1)
    assert int(nan_rows.sum().item()) == ref
    assert torch.isfinite(out[~nan_rows]).all()
    assert torch.isnan(nrm[nan_rows]).all() and torch.isfinite(nrm[~nan_rows]).all()
    assert (nrm[~nan_rows].norm(dim=1) - 1).abs().max().item() < 1e-5
    # a direction and its copies scaled by 2^e, -140 <= e <= 120, give the
    # same bits: components on a 2^-9 grid stay exact down to subnormals
    q = np.round(workloads.uniform_dirs(4096, rng) * 512.0) / 512.0
    q = q[np.abs(q).max(axis=1) > 0].astype(np.float32)
    base = torch.as_tensor(q).to(DEV)
    n = base.shape[0]
    o1 = torch.empty((n, 4), device=DEV)
    shm.shm_query_value_grad(lut, shm.SHM_F32, shm.SHM_LAYOUT_TEXEL, 8, 1, base, n, o1)
    assert torch.isfinite(o1).all()
    for e in (-140, -130, -100, -64, -30, 30, 64, 100, 120):
        sc = (q.astype(np.float64) * 2.0 ** e).astype(np.float32)
        assert (sc.astype(np.float64) * 2.0 ** -e == q).all()  # exact
        o2 = torch.empty((n, 4), device=DEV)
        shm.shm_query_value_grad(lut, shm.SHM_F32, shm.SHM_LAYOUT_TEXEL, 8, 1, torch.as_tensor(sc).to(DEV), n, o2)
        assert torch.equal(o1.view(torch.int32), o2.view(torch.int32)), e
    assert c.item() == ref + int((~(np.isfinite(d[:1000]).all(axis=1) & (np.abs(d[:1000]).max(axis=1) > 0))).sum())


@pytest.mark.parametrize("dt", [torch.float32, torch.float16])
def test_gather_footprints_bit_exact(dt):
    """Step a3 alone: every query's 16 footprint scalars, for both layouts,
    equal the LUT's texels at the query's cell (cell keys, themselves checked
    against the oracle's FP64 decision up to counted ties), corner by corner; FP16 data
    decode exactly; NaN for invalid directions.  3 objects, a ragged count."""
    rng = np.random.default_rng(21)
    N, n_obj, qpo = 9, 3, 1001
    lut = torch.as_tensor(workloads.random_lut(N, rng, n_obj=n_obj)).to(DEV, dt).contiguous()
    d = workloads.uniform_dirs(n_obj * qpo, rng)
    d[7] = 0.0
    d[500, 1] = np.nan
    dirs = torch.as_tensor(d).to(DEV)
    keys = shm.cell_keys(N, dirs, n_obj=n_obj).cpu().numpy().astype(np.int64)
    tex = lut.float().cpu().numpy()
    ok = keys >= 0
    assert (~ok).sum() == 2
    i0 = keys[ok] % (N + 1)
    j0 = (keys[ok] // (N + 1)) % (N + 1)
    f = (keys[ok] // (N + 1) ** 2) % 6
    o = keys[ok] // ((N + 1) ** 2 * 6)
    ref = np.stack([tex[o, f, j0 + dj, i0 + di] for dj, di in ((0, 0), (0, 1), (1, 0), (1, 1))], axis=1)
    layouts = [(shm.SHM_LAYOUT_TEXEL, lut), (shm.SHM_LAYOUT_CELL, shm.to_cells(lut))]
    for layout, src in layouts:
        foot = torch.empty((n_obj * qpo, 4, 4), device=DEV)
        code = shm.SHM_F16 if dt == torch.float16 else shm.SHM_F32
        shm.shm_gather_footprints(src, code, layout, N, n_obj, dirs, qpo, foot)
        got = foot.cpu().numpy()
        assert np.isnan(got[~ok]).all()
        assert np.array_equal(got[ok], ref), layout


def test_f16_cells_from_f32_data():
    """FP16 cells made from FP32 cells (shm_cells_to_f16): (1) the encoding
    bit for bit (corner 0 rounded once; corners 1..3 with r replaced by its
    FP32 difference from corner 0's r, rounded once); (2) the FP16 cell query
    gives the bits of the FP32 cell query on the decoded cells; (3) against
    the oracle (FP64, on the FP32 LUT) its gradient error is far below that of
    plain FP16 texels: the value's rounding no longer enters the derivatives."""
    c = workloads.sh_glyph_coeffs(8, 1, rng(31))[0]
    N = 32
    lut = oracle.bake_sh(c, N).astype(np.float32)
    cells32 = shm.to_cells(gpu(lut)[None])
    c16 = shm.cells_to_f16(cells32)
    src = cells32.cpu().numpy().reshape(-1, 4, 4)
    enc = src.copy()
    enc[:, 1:, 0] = enc[:, 1:, 0] - enc[:, :1, 0]
    assert np.array_equal(c16.cpu().numpy().reshape(-1, 4, 4).view(np.uint16), enc.astype(np.float16).view(np.uint16))
    dirs = workloads.uniform_dirs(65536, rng(32))
    d = gpu(dirs)
    o16 = shm.query(c16, d, layout=shm.SHM_LAYOUT_CELL)
    dec = gpu(decode_f16_cells(c16.cpu().numpy()))
    o32d = shm.query(dec, d, layout=shm.SHM_LAYOUT_CELL)
    torch.cuda.synchronize()
    assert torch.equal(o16.view(torch.int32), o32d.view(torch.int32))
    ref = oracle.query(lut.astype(np.float64), dirs)
    plain = gpu_query(lut.astype(np.float16).astype(np.float32), dirs, shm.SHM_LAYOUT_TEXEL, dtype=torch.float16)

    def grad_err(o):
        g, gr = o[:, 1:], ref[:, 1:]
        gn = np.linalg.norm(gr, axis=1)
        return np.linalg.norm(g - gr, axis=1) / np.maximum(gn, np.sqrt(np.mean(gn ** 2)))

    e16, ep = grad_err(o16.cpu().numpy()), grad_err(plain)
    print(f"FP16 gradient error, max / rms: delta cells {e16.max():.3g} / {np.sqrt(np.mean(e16**2)):.3g}, "
          f"plain texels {ep.max():.3g} / {np.sqrt(np.mean(ep**2)):.3g}")
    assert e16.max() < 0.05 * ep.max() and e16.max() < 5e-3
    v16 = np.abs(o16.cpu().numpy()[:, 0] - ref[:, 0]) / np.abs(ref[:, 0])
    assert v16.max() < 1e-3  # FP16 value rounding, as before
