"""Rendered radius on the GPU (Sec. 3.1): scaled and signed queries, the |r|
bound, and the trace with sign tracking and the adaptive bisection budget,
against the FP64 oracle on the same LUT data."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2602_20063_amd as shm
import workloads
from parity import angle_deg, check_value_grad

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def gpu(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def check_signed(out, ref, what, s):
    """Values: |dR| <= 1e-5 max(|R_ref|, RMS R_ref) (R = s|r| reaches 0 on
    the zero set of r).  Gradients and normals only where |r| is clear of
    0: there grad R = s sign(r) grad r jumps, and FP32 and FP64 may take the
    sign of an r within rounding of 0 differently."""
    ok = np.isfinite(ref[:, 0])
    assert np.array_equal(ok, np.isfinite(out[:, 0])), what
    o, r = out[ok], ref[ok]
    rms = np.sqrt(np.mean(r[:, 0] ** 2))
    dv = np.abs(o[:, 0] - r[:, 0]) / np.maximum(np.abs(r[:, 0]), rms)
    assert dv.max() <= 1e-5, (what, dv.max())
    clear = ok & (np.abs(ref[:, 0]) > 1e-4 * s)
    check_value_grad(out[clear], ref[clear], what, val_rtol=np.inf)  # values checked above
    return clear


def signed_lut(N, seed):
    """A signed SH function: z (two lobes of opposite sign) plus a small
    L = 4 perturbation, baked analytically."""
    r = np.random.default_rng(seed)
    c = 0.08 * r.standard_normal(25)
    c[0] = 0.0
    c[2] += math.sqrt(4 * math.pi / 3)
    return oracle.bake_sh(c, N).astype(np.float32)


@pytest.mark.parametrize("layout", [shm.SHM_LAYOUT_TEXEL, shm.SHM_LAYOUT_CELL])
@pytest.mark.parametrize("signed", [False, True])
def test_query_scaled_matches_oracle(layout, signed):
    N, s = 20, 0.7
    lut = signed_lut(N, 5)
    dirs = workloads.uniform_dirs(40000, np.random.default_rng(6))
    dirs[11] = 0.0
    lt = gpu(lut)
    if layout == shm.SHM_LAYOUT_CELL:
        lt = shm.to_cells(lt[None])
    out, n, sg = shm.query_scaled(lt, gpu(dirs), scale=s, signed=signed, layout=layout)
    torch.cuda.synchronize()
    out, n, sg = out.cpu().numpy(), n.cpu().numpy(), sg.cpu().numpy()
    ref, rn, rs = oracle.query_scaled(lut.astype(np.float64), dirs, scale=s, signed=signed)
    ok = np.isfinite(ref[:, 0])
    assert np.isnan(out[~ok]).all() and (sg[~ok] == 0).all()
    clear = check_signed(out, ref, f"scaled signed={signed}", s)
    assert np.array_equal(sg[clear], rs[clear])
    ang = angle_deg(n[clear], rn[clear])
    assert np.median(ang) < 1e-4 and np.quantile(ang, 0.999) < 0.05, (np.median(ang), ang.max())
    if signed:
        assert (out[ok, 0] >= 0).all() and (sg[ok] < 0).mean() > 0.3


def test_query_scaled_fp16():
    N, s = 16, 1.3
    lut16 = signed_lut(N, 7).astype(np.float16)
    dirs = workloads.uniform_dirs(20000, np.random.default_rng(8))
    out, _, sg = shm.query_scaled(gpu(lut16, torch.float16), gpu(dirs), scale=s, signed=True)
    torch.cuda.synchronize()
    ref, _, rs = oracle.query_scaled(lut16.astype(np.float64), dirs, scale=s, signed=True)
    clear = check_signed(out.cpu().numpy(), ref, "scaled fp16", s)
    assert np.array_equal(sg.cpu().numpy()[clear], rs[clear])


def test_lut_rmax_signed_bound():
    lut = signed_lut(24, 9)
    g = shm.lut_rmax(gpu(lut), signed=True).item()
    ref = oracle.rmax_bound(lut.astype(np.float64), absval=True)
    assert abs(g - ref) <= 1e-6 * ref
    # max |c| over the control points = max(max c, max -c), exactly
    plain, plain_neg = shm.lut_rmax(gpu(lut)).item(), shm.lut_rmax(gpu(-lut)).item()
    assert plain < g or plain_neg < g
    assert max(plain, plain_neg) == g
    assert shm.lut_rmax(gpu(-lut), signed=True).item() == g


def test_trace_signed_adaptive_matches_oracle():
    N, s = 32, 0.6
    lut = signed_lut(N, 10)
    rmax = s * oracle.rmax_bound(lut.astype(np.float64), absval=True) * 1.0001
    o, d = workloads.camera_rays(160, 120, eye=(1.5, 0.4, 0.6), vfov_deg=45.0)
    px = 60 / math.tan(math.radians(22.5))  # focal length of a 120-pixel-high image
    tg, og, ng, sg, eg = shm.trace_ex(gpu(lut), (0.0, 0.0, 0.0), rmax, gpu(o), gpu(d), scale=s, signed=True,
                                      px_per_unit=px, eps_px=0.125)
    torch.cuda.synchronize()
    tg, og, ng, sg, eg = (x.cpu().numpy() for x in (tg, og, ng, sg, eg))
    tr, orf, nr, sr, er = oracle.trace_ex(lut.astype(np.float64), np.zeros(3), np.float32(rmax), o, d, scale=s,
                                          signed=True, px=px, eps_px=0.125)
    hg, hr = np.isfinite(tg), np.isfinite(tr)
    assert 0.1 < hr.mean() < 0.9
    assert np.mean(hg != hr) <= 0.002
    both = hg & hr
    rel = np.abs(tg[both] - tr[both]) / tr[both]
    assert np.median(rel) < 1e-6 and np.mean(rel < 1e-4) > 0.995
    ang = angle_deg(ng[both], nr[both])
    assert np.median(ang) < 1e-3 and np.mean(ang < 0.05) > 0.995
    # sign of r at the hit, away from the r = 0 kink
    clear = both & (np.abs(orf[:, 0]) > 1e-3)
    assert np.array_equal(sg[clear], sr[clear]) and (sr[clear] < 0).any() and (sr[clear] > 0).any()
    assert (sg[~hg] == 0).all()
    # every ray of one camera gets the same budget; evaluations agree
    k = oracle.bisect_budget(o[0], np.zeros(3), np.float32(rmax), px, 0.125, 20, 16)
    assert 0 < k < 16
    assert np.mean(eg == er) > 0.995
    march = eg[hg].astype(int) - k - 3 - 1
    assert ((march >= 1) & (march <= 20)).all()


def test_trace_budget_bit_exact():
    """The per-ray bisection count is the FP32 decision of the oracle for
    every origin.  Two march samples, rays aimed just off the centre of a
    constant sphere: the first sample (nearest the centre) is always inside,
    so evaluations = 1 + budget + Newton + 1."""
    N = 4
    lut = np.zeros((6, N + 2, N + 2, 4), np.float32)
    lut[..., 0] = 0.8
    r = np.random.default_rng(11)
    P = 20000
    dirn = r.standard_normal((P, 3))
    dirn /= np.linalg.norm(dirn, axis=1, keepdims=True)
    dist = np.exp(r.uniform(math.log(1.5), math.log(5000.0), P))
    o = (dirn * dist[:, None]).astype(np.float32)
    aim = r.uniform(-0.05, 0.05, (P, 3))
    d = (aim - o).astype(np.float32)
    px, eps = 1234.5, 0.1
    tg, _, _, _, eg = shm.trace_ex(gpu(lut), (0.0, 0.0, 0.0), 0.85, gpu(o), gpu(d), px_per_unit=px, eps_px=eps,
                                   n_march=2, n_bisect=40, n_newton=2, normals=False)
    torch.cuda.synchronize()
    tg, eg = tg.cpu().numpy(), eg.cpu().numpy().astype(int)
    assert np.isfinite(tg).all()
    ref = np.array([oracle.bisect_budget(o[i], np.zeros(3), 0.85, px, eps, 2, 40) for i in range(P)])
    assert len(set(ref.tolist())) > 10
    np.testing.assert_array_equal(eg - 1 - 2 - 1, ref)
