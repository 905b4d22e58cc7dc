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
