"""The memory probes (shm_probe.h) compute what they claim: on a LUT region
filled with ones, a request that reads req_bytes adds req_bytes / 16 to each
of the four result components, on top of its own direction when it streams
directions; every request writes its own result row."""
import numpy as np
import pytest
import torch

import paper_2602_20063_amd as shm

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("req", [0, 16, 32, 64, 128])
def test_probe_gather_results(req):
    n_regions, per_region, region = 37, 300, 4096  # ragged: 300 requests per region, two workgroups
    Q = n_regions * per_region
    base = torch.ones(n_regions * region // 4, device=DEV)
    dirs = torch.as_tensor(np.random.default_rng(3).standard_normal((Q, 3)).astype(np.float32)).to(DEV)
    out = torch.full((Q, 4), float("nan"), device=DEV)
    shm.shm_probe_gather(base, region, n_regions, per_region, req, 7, shm.SHM_PROBE_DIRS | shm.SHM_PROBE_OUT, dirs, out)
    k = req // 16
    expect = torch.cat([dirs, torch.zeros((Q, 1), device=DEV)], dim=1)
    for _ in range(k):  # the probe adds one float4 of ones at a time (FP32, in order)
        expect = expect + 1.0
    torch.cuda.synchronize()
    assert torch.equal(out, expect)
    # results only (no direction stream)
    out.fill_(float("nan"))
    shm.shm_probe_gather(base, region, n_regions, per_region, req, 7, shm.SHM_PROBE_OUT, None, out)
    torch.cuda.synchronize()
    assert torch.equal(out, torch.full_like(out, float(k)))


def test_probe_sinks_are_not_written():
    base = torch.ones(1 << 16, device=DEV)
    sink = torch.full((4,), 123.0, device=DEV)
    shm.shm_probe_gather(base, 4096, 64, 256, 64, 1, 0, None, sink)
    shm.shm_probe_stream_read(base, base.numel() * 4, sink)
    torch.cuda.synchronize()
    assert torch.equal(sink, torch.full_like(sink, 123.0))


@pytest.mark.parametrize("wps,chains", [(1, 1), (2, 4), (4, 8)])
def test_mfma_probe_counts_its_flops(wps, chains):
    """The matrix-core probe reports 2,048 flops per MFMA for 4 waves per
    workgroup, wps workgroups per compute unit, `iters` rounds of `chains`
    MFMAs, leaves its sink alone, and runs at a plausible rate (between 1
    and 200 TFLOP/s: FP32 matrix peak 157.3)."""
    sink = torch.full((4,), 7.0, device=DEV)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    iters = 2000
    shm.shm_probe_mfma_f32(wps, chains, iters, sink)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    flops = shm.shm_probe_mfma_f32(wps, chains, iters, sink)
    e1.record()
    e1.synchronize()
    assert flops == n_cu * wps * 4 * iters * chains * 2048
    assert torch.equal(sink, torch.full_like(sink, 7.0))
    tf = flops / (e0.elapsed_time(e1) * 1e-3) / 1e12
    print(f"wps {wps} chains {chains}: {tf:.1f} TFLOP/s")
    assert 1.0 < tf < 200.0


@pytest.mark.parametrize("dtype,layout", [(shm.SHM_F32, shm.SHM_LAYOUT_CELL), (shm.SHM_F16, shm.SHM_LAYOUT_CELL),
                                          (shm.SHM_F32, shm.SHM_LAYOUT_TEXEL), (shm.SHM_F16, shm.SHM_LAYOUT_TEXEL)])
def test_plan_probe_walks_every_query_of_its_object(dtype, layout):
    """The plan probe answers every query of the plan once, from its own
    object's LUT: each object's LUT holds one distinct 32-bit word, so the
    footprint's word sum names the object, in every launch shape."""
    Ns, Qs = [5, 8, 3, 1], [700, 131, 2000, 64]
    cell = layout == shm.SHM_LAYOUT_CELL
    elems = [6 * (N + 1) ** 2 * 16 if cell else 6 * (N + 2) ** 2 * 4 for N in Ns]
    offs = np.concatenate([[0], np.cumsum(elems)[:-1]])
    qb = np.concatenate([[0], np.cumsum(Qs)[:-1]])
    Q = int(sum(Qs))
    f16 = dtype == shm.SHM_F16
    vals = [1.5, -2.25, 3.0, 0.125]
    lut = torch.empty(int(sum(elems)), dtype=torch.float16 if f16 else torch.float32, device=DEV)
    words = []
    for o, v in enumerate(vals):
        lut[int(offs[o]):int(offs[o]) + elems[o]] = v
        b = int(np.array([v], np.float16 if f16 else np.float32).view(np.uint16 if f16 else np.uint32)[0])
        words.append(b | (b << 16) if f16 else b)
    n_words = 8 if f16 else 16  # 32 B (FP16) or 64 B (FP32) per footprint, both layouts
    expect_w = np.concatenate([np.full(q, (n_words * w) & 0xFFFFFFFF, np.uint32) for q, w in zip(Qs, words)])
    dirs = torch.as_tensor(np.random.default_rng(9).standard_normal((Q, 3)).astype(np.float32)).to(DEV)
    plan = shm.Plan([(int(offs[o]), Ns[o], int(qb[o]), Qs[o]) for o in range(4)], dtype, layout)
    try:
        for shape in [(256, 2, 512, 4), (64, 1, 64, 2), (128, 4, 1024, 1), (256, 1, 256, 0), (64, 2, 128, 0),
                      (128, 4, 512, 0)]:
            plan.set_shape(*shape)
            out = torch.full((Q, 4), float("nan"), device=DEV)
            plan.probe(lut, dirs, out, seed=11)
            torch.cuda.synchronize()
            assert torch.equal(out[:, :3], dirs), shape
            got_w = out[:, 3].contiguous().view(torch.int32).cpu().numpy().view(np.uint32)
            assert np.array_equal(got_w, expect_w), shape
    finally:
        plan.close()
