"""Parity at the benchmark sizes, in the launch configurations bench.py times,
on sampled outputs the oracle computes one by one (or through properties
that hold at any size):
  * SH glyph field: 32,768 glyphs, L = 8, N = 32, 8,388,608 queries, cell
    layout, FP32;
  * bump impostor trace: N = 256, 1920 x 1080 rays;
  * backward: N = 512, 2^22 queries (three radix passes);
  * uneven batch: 4,096 objects, ~10^8 queries, FP16 cell LUTs, one
    autotuned graph-captured persistent launch.
Every oracle evaluation uses the LUT values the GPU produced (so the query,
trace and backward are compared on the same data) and the bake is checked
separately on the sampled objects."""
import numpy as np
import pytest
import torch

import bench
import oracle
import paper_2602_20063_amd as shm
import workloads
from parity import check_value_grad, decode_f16_cells
from test_gpu_bake import check_lut
from test_gpu_trace import compare

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def spread(n, k, rng):
    """k sample indices over range(n), both ends included."""
    idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, k - 2, replace=False)]))
    return np.sort(idx)


def test_glyph_field_full_size_sampled():
    W = bench.W2
    n, L, N, qp = W["n_glyph"], W["L"], W["N"], W["q_per"]
    c, dirs = bench.setup_w2()
    c_t, d_t = torch.as_tensor(c).to(DEV), torch.as_tensor(dirs).to(DEV)
    lut = shm.bake_sh(c_t, N)
    cells = shm.to_cells(lut)
    out = torch.empty((n * qp, 4), device=DEV)
    shm.shm_query_value_grad(cells, shm.SHM_F32, shm.SHM_LAYOUT_CELL, N, n, d_t, qp, out)
    torch.cuda.synchronize()
    g = spread(n, 48, np.random.default_rng(1))
    lut_s = lut[torch.as_tensor(g, device=DEV)].cpu().numpy()
    check_lut(lut_s, oracle.bake_sh(c[g].astype(np.float64), N), "glyph-field bake, sampled glyphs")
    rows = (g[:, None] * qp + np.arange(qp)[None, :]).reshape(-1)
    per = lut_s[0].size // 4
    ref = oracle.query_objects(lut_s.reshape(-1).astype(np.float64), np.arange(len(g)) * per, [N] * len(g),
                               np.arange(len(g)) * qp, [qp] * len(g), dirs[rows])
    got = out[torch.as_tensor(rows, device=DEV)].cpu().numpy()
    check_value_grad(got, ref, "glyph field, sampled glyphs")


def test_trace_full_size_sampled():
    N = 256
    mu, amp, width = workloads.bump_params(workloads.rng_for(3))
    md = shm.margin_dirs(N).cpu().numpy().reshape(-1, 3)
    samples = workloads.bumps_value(mu, amp, width, 1.0, md).astype(np.float32)
    lut = shm.bake_fd(torch.as_tensor(samples).to(DEV), N)
    rmax = float(shm.lut_rmax(lut).item()) * 1.0001
    o, d = workloads.camera_rays(1920, 1080)
    t, out, nrm = shm.trace(lut, (0.0, 0.0, 0.0), rmax, torch.as_tensor(o).to(DEV), torch.as_tensor(d).to(DEV))
    torch.cuda.synchronize()
    k = spread(o.shape[0], 4000, np.random.default_rng(2))
    ref = oracle.trace(lut[0].cpu().numpy().astype(np.float64), np.zeros(3), rmax, o[k], d[k])
    compare((t.cpu().numpy()[k], out.cpu().numpy()[k], nrm.cpu().numpy()[k]), ref, "trace 1920x1080")
    assert 0.2 < np.isfinite(ref[0]).mean() < 0.8


def test_backward_full_size():
    """2^22 queries at N = 512.  dL/dLUT through the adjoint identity (the
    outputs are linear in the LUT): sum(grad_lut * D) = sum(g * query(D)) for
    a random LUT-shaped D, with the forward itself checked elsewhere; dL/d
    dirs against the oracle on sampled queries."""
    N, Q = 512, 1 << 22
    r = workloads.rng_for(4)
    dirs = workloads.uniform_dirs(Q, r)
    lut_np = workloads.random_lut(N, r)
    d_t, lut = torch.as_tensor(dirs).to(DEV), torch.as_tensor(lut_np).to(DEV)
    gen = torch.Generator(device=DEV).manual_seed(4)
    g = torch.randn((Q, 4), device=DEV, generator=gen)
    D = torch.randn(lut.shape, device=DEV, generator=gen)
    bc = shm.BackwardContext(N, 1, d_t, Q)
    gl, gd = bc.backward(lut, g)
    fD = shm.query(D[None], d_t)
    torch.cuda.synchronize()
    lhs = (gl.double() * D.double()).sum().item()
    rhs = (g.double() * fD.double()).sum().item()
    scale = (gl.double() * D.double()).abs().sum().item()
    assert abs(lhs - rhs) <= 1e-5 * scale, (lhs, rhs, scale)
    k = spread(Q, 3000, np.random.default_rng(3))
    _, rd = oracle.backward(lut_np, dirs[k], g.cpu().numpy()[k])
    gk = gd.cpu().numpy()[k]
    gn = np.linalg.norm(rd, axis=1)
    floor = np.sqrt(np.mean(gn ** 2))
    _e = np.linalg.norm(gk - rd, axis=1) / np.maximum(gn, floor)
    print('grad_dirs error max %.3e rms %.3e' % (_e.max(), np.sqrt(np.mean(_e ** 2))))
    assert _e.max() < 2e-5  # FP32 vs FP64 (measured <= 1e-6)


def test_backward_full_size_texels_elementwise_and_fd():
    """The fitting workload's backward at full size (N = 512, 2^22 directions
    sorted by cell, as bench.py runs it), dL/dLUT texel by texel on 64
    sampled texels x 4 channels (gutter corners and edges included):
      * against the oracle's backward over the queries whose cells touch a
        sampled texel (no other query reads it, so this is the full sum);
      * against central differences of the FP64 loss sum(g * query(LUT)) in
        the same texel (the loss changes only through those queries)."""
    N, Q = 512, 1 << 22
    r = workloads.rng_for(4)
    dirs_t = torch.as_tensor(workloads.uniform_dirs(Q, r)).to(DEV)
    dirs_t = dirs_t[torch.argsort(shm.cell_keys(N, dirs_t).to(torch.int64) & 0xFFFFFFFF, stable=True)].contiguous()
    dirs = dirs_t.cpu().numpy()
    lut_np = workloads.random_lut(N, np.random.default_rng(44))
    lut = torch.as_tensor(lut_np).to(DEV)[None].contiguous()
    g_t = torch.randn((Q, 4), device=DEV, generator=torch.Generator(device=DEV).manual_seed(44))
    bc = shm.BackwardContext(N, 1, dirs_t, Q)
    gl = bc.backward(lut, g_t, want_dirs=False)[0][0].cpu().numpy()
    g = g_t.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(45)
    P = N + 2
    tex = [(f, q, p) for f in (0, 3, 5) for (q, p) in ((0, 0), (0, P - 1), (P - 1, 0), (P - 1, P - 1))]
    tex += [(int(rng.integers(6)), 0, int(rng.integers(1, P - 1))) for _ in range(6)]      # gutter rows
    tex += [(int(rng.integers(6)), int(rng.integers(1, P - 1)), P - 1) for _ in range(6)]  # gutter columns
    while len(tex) < 64:
        tex.append((int(rng.integers(6)), int(rng.integers(1, P - 1)), int(rng.integers(1, P - 1))))
    face, i0, j0, _, _ = oracle.locate(dirs, N)
    C = N + 1
    key = (face.astype(np.int64) * C + j0) * C + i0
    key[face < 0] = -1

    def touching(f, q, p):
        cells = [(f * C + jj) * C + ii for jj in (q - 1, q) for ii in (p - 1, p) if 0 <= jj <= N and 0 <= ii <= N]
        return np.flatnonzero(np.isin(key, cells))

    sel = [touching(*t) for t in tex]
    union = np.unique(np.concatenate(sel))
    rl, _ = oracle.backward(lut_np, dirs[union], g[union], want_dirs=False)
    lut64 = lut_np.astype(np.float64)
    got, ref, fd = [], [], []
    for t, idx in zip(tex, sel):
        for ch in range(4):
            got.append(gl[t + (ch,)])
            ref.append(rl[t + (ch,)])
            if idx.size == 0:
                fd.append(0.0)
                continue
            eps = 1e-3
            keep = lut64[t + (ch,)]
            lut64[t + (ch,)] = keep + eps
            lp = np.sum(oracle.query(lut64, dirs[idx]) * g[idx])
            lut64[t + (ch,)] = keep - eps
            lm = np.sum(oracle.query(lut64, dirs[idx]) * g[idx])
            lut64[t + (ch,)] = keep
            fd.append((lp - lm) / (2 * eps))
    got, ref, fd = (np.array(x).reshape(-1, 4) for x in (got, ref, fd))
    counts = np.array([x.size for x in sel])
    print(f"sampled texels: {len(tex)}, queries per texel {counts.min()}..{counts.max()} (mean {counts.mean():.1f})")
    # gutter corners are read only by queries within half a cell of a cube
    # corner (mostly none); the other samples are mostly read
    assert (counts[12:] > 0).sum() >= 48, counts
    scale = np.sqrt(np.mean(ref ** 2, axis=0))  # per channel
    e_ref = np.abs(got - ref) / np.maximum(np.abs(ref), scale)
    e_fd = np.abs(fd - ref) / np.maximum(np.abs(ref), scale)
    e_gfd = np.abs(got - fd) / np.maximum(np.abs(fd), scale)
    print(f"grad_lut vs oracle: max rel {e_ref.max():.2e}; vs FD {e_gfd.max():.2e}; oracle vs FD {e_fd.max():.2e}")
    assert e_ref.max() < 1e-5 and e_gfd.max() < 1e-5  # FP32 sums vs FP64 (measured 4.4e-7)
    assert e_fd.max() < 1e-7


def test_uneven_batch_full_size_sampled(tmp_path):
    B = bench.build_uneven_batch()
    objs, n_obj, Qtot = B["objs"], B["n_obj"], B["Qtot"]
    lut16 = shm.cells_to_f16(B["lut32"])
    out = torch.full((Qtot, 4), float("nan"), device=DEV)
    plan = shm.Plan(objs, shm.SHM_F16, shm.SHM_LAYOUT_CELL)
    plan.autotune(lut16, B["dirs"], out, cache_path=str(tmp_path / "tune.json"))
    out.fill_(float("nan"))
    plan.capture_graph(lut16, B["dirs"], out)
    plan.graph_launch()
    torch.cuda.synchronize()
    plan.close()
    spec = B["spec"]
    rng = np.random.default_rng(5)
    big = np.flatnonzero(spec["N"] == spec["N"].max())
    sel = np.unique(np.concatenate([spread(n_obj, 30, rng), big[:4], [int(np.argmax(spec["Q"]))]]))
    # each sampled object: the FP32 cell query on its decoded FP16 cells gives
    # the batch's bits (the FP32 cell query is checked against the oracle
    # elsewhere), and stays within the FP16 error of the FP32 data
    for o in sel:
        off, Nn, q0, q = objs[o]
        n = shm.shm_lut_elems(Nn, shm.SHM_LAYOUT_CELL)
        dec = torch.as_tensor(decode_f16_cells(lut16[off:off + n].cpu().numpy())).to(DEV)
        ref = torch.empty((q, 4), device=DEV)
        shm.shm_query_value_grad(dec, shm.SHM_F32, shm.SHM_LAYOUT_CELL, Nn, 1, B["dirs"][q0:q0 + q], q, ref)
        torch.cuda.synchronize()
        assert torch.equal(out[q0:q0 + q].view(torch.int32), ref.view(torch.int32)), o
    q_all = out[:, 0]
    assert torch.isfinite(q_all).all()
    # the plan-free object query (device descriptors) gives the plan's bits
    out2 = torch.full((Qtot, 4), float("nan"), device=DEV)
    shm.query_objects(lut16, B["dirs"], objs, layout=shm.SHM_LAYOUT_CELL, out=out2)
    torch.cuda.synchronize()
    assert torch.equal(out2.view(torch.int32), out.view(torch.int32))


def test_trace_full_size_bound_map_same_bits():
    """The benchmark's trace with the bound map and image tiles gives the
    bits of the plain launch (1920 x 1080, N = 256)."""
    N = 256
    mu, amp, width = workloads.bump_params(workloads.rng_for(3))
    md = shm.margin_dirs(N).cpu().numpy().reshape(-1, 3)
    samples = workloads.bumps_value(mu, amp, width, 1.0, md).astype(np.float32)
    lut = shm.bake_fd(torch.as_tensor(samples).to(DEV), N)
    rmax = float(shm.lut_rmax(lut).item()) * 1.0001
    o, d = workloads.camera_rays(1920, 1080)
    og, dg = torch.as_tensor(o).to(DEV), torch.as_tensor(d).to(DEV)
    a = shm.trace(lut, (0.0, 0.0, 0.0), rmax, og, dg)
    b = shm.trace(lut, (0.0, 0.0, 0.0), rmax, og, dg, image_width=1920, bound_map=shm.lut_bound_map(lut))
    for x, y in zip(a, b):
        assert torch.equal(x.view(torch.int32), y.view(torch.int32))


def test_fit_step_full_size():
    """The fitting workload's one-kernel step (N = 512, 2^22 directions
    sorted by cell, as bench.py runs it) against the three-kernel step, two
    steps from a random LUT: the Adam moments (linear in the gradients)
    within 1e-5 of their largest; the parameters within 1e-6 except where the
    second gradient nearly cancels the first in m, so that m/sqrt(v) turns
    rounding-level differences into visible ones (a handful of the 6.3 M
    texels), and never further apart than two Adam steps (2 lr); every
    interior texel moved."""
    N, Q = 512, 1 << 22
    r = workloads.rng_for(4)
    dirs = torch.as_tensor(workloads.uniform_dirs(Q, r)).to(DEV)
    dirs = dirs[torch.argsort(shm.cell_keys(N, dirs).to(torch.int64) & 0xFFFFFFFF, stable=True)].contiguous()
    lut = torch.as_tensor(workloads.random_lut(N, r)).to(DEV)[None].contiguous()
    tv, tg = workloads.fbm_target_torch(dirs, seed=5)
    w = dirs / dirs.norm(dim=1, keepdim=True)
    tn = tv.float()[:, None] * w - tg.float()
    tn = (tn / tn.norm(dim=1, keepdim=True)).contiguous()
    tv = tv.float().contiguous()
    a = shm.LutFit(lut.clone(), dirs, tv, tn, w_value=1000.0, lr_value=1e-3, lr_deriv=3e-4, fused=True)
    b = shm.LutFit(lut.clone(), dirs, tv, tn, w_value=1000.0, lr_value=1e-3, lr_deriv=3e-4, fused=False)
    for step in (1, 2):
        a.step()
        b.step()
        torch.cuda.synchronize()
        dm = (a.m - b.m).abs().max().item()
        assert dm <= 1e-5 * b.m.abs().max().item(), (step, dm)
        dp = (a.lut - b.lut).abs()
        far = int((dp > 1e-6).sum().item())
        print(f"step {step}: max |dp| {dp.max().item():.3g}, {far} texel channels beyond 1e-6")
        assert far <= 1e-5 * dp.numel() and dp.max().item() <= 2 * 1e-3, (step, far)
    moved = (a.lut != lut)[0, :, 1:N + 1, 1:N + 1].float().mean().item()
    assert moved > 0.999, moved


def decode_cells_gpu(c16):
    """The FP32 cells FP16 cells decode to (FP32 additions, on the GPU)."""
    c = c16.float().reshape(-1, 4, 4)
    c[:, 1:, 0] += c[:, :1, 0]
    return c.reshape(c16.shape)


def test_glyph_field_f16_cells_full_size():
    """The benchmark's FP16 cell form (32,768 glyphs, N = 32, 8,388,608
    queries; cells made from the FP32 cells) gives the bits of the FP32 cell
    query on the cells it decodes to, for every query."""
    W = bench.W2
    n, N, qp = W["n_glyph"], W["N"], W["q_per"]
    c, dirs = bench.setup_w2()
    d_t = torch.as_tensor(dirs).to(DEV)
    cells = shm.to_cells(shm.bake_sh(torch.as_tensor(c).to(DEV), N))
    c16 = shm.cells_to_f16(cells)
    del cells
    dec = decode_cells_gpu(c16)
    a = torch.empty((n * qp, 4), device=DEV)
    b = torch.empty((n * qp, 4), device=DEV)
    shm.shm_query_value_grad(c16, shm.SHM_F16, shm.SHM_LAYOUT_CELL, N, n, d_t, qp, a)
    shm.shm_query_value_grad(dec, shm.SHM_F32, shm.SHM_LAYOUT_CELL, N, n, d_t, qp, b)
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_trace_f16_cells_full_size():
    """The benchmark's FP16-cell trace (1920 x 1080, N = 256, 8 x 8 tiles,
    the bound map of the FP16 cells) gives the bits of the FP32-cell trace
    of the decoded cells with that one's own bound map."""
    N = 256
    mu, amp, width = workloads.bump_params(workloads.rng_for(3))
    md = shm.margin_dirs(N).cpu().numpy().reshape(-1, 3)
    samples = workloads.bumps_value(mu, amp, width, 1.0, md).astype(np.float32)
    c16 = shm.cells_to_f16(shm.to_cells(shm.bake_fd(torch.as_tensor(samples).to(DEV), N)))
    dec = decode_cells_gpu(c16)
    rmax = float(shm.lut_rmax(c16[0]).item()) * 1.0001
    assert float(shm.lut_rmax(dec[0]).item()) * 1.0001 == rmax
    o, d = workloads.camera_rays(1920, 1080)
    og, dg = torch.as_tensor(o).to(DEV), torch.as_tensor(d).to(DEV)
    a = shm.trace(c16[0], (0.0, 0.0, 0.0), rmax, og, dg, image_width=1920, bound_map=shm.lut_bound_map(c16[0]))
    b = shm.trace(dec[0], (0.0, 0.0, 0.0), rmax, og, dg, image_width=1920, bound_map=shm.lut_bound_map(dec[0]))
    for x, y in zip(a, b):
        assert torch.equal(x.view(torch.int32), y.view(torch.int32))
    assert 0.2 < torch.isfinite(a[0]).float().mean().item() < 0.8
