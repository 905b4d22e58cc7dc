"""The size limits of the entry points on the GPU against the oracle: face
size 1 and the largest face (1,024), SH order 16; sampled where the whole
oracle result would take long."""
import numpy as np
import pytest
import torch

import oracle
import paper_2602_20063_amd as shm
import workloads
from test_gpu_bake import check_lut
from test_gpu_trace import compare

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def sample_texels(N, k, rng):
    """k padded texels (face, q, p), the gutter corners of every face included."""
    P = N + 2
    f = rng.integers(0, 6, k)
    q = rng.integers(0, P, k)
    p = rng.integers(0, P, k)
    corners = np.array([(fc, a, b) for fc in range(6) for a in (0, P - 1) for b in (0, P - 1)])
    return np.concatenate([corners, np.stack([f, q, p], axis=1)])


@pytest.mark.parametrize("L,N", [(8, 1024), (16, 300), (2, 1), (16, 1)])
def test_bake_extreme_sizes(L, N):
    """The register-resident contraction at the largest face, the LDS-staged
    one at SH order 16, and face size 1, on sampled texels (gutter corners
    included) against the oracle's bake at those texel centres."""
    rng = np.random.default_rng(L * 7 + N)
    c = workloads.sh_glyph_coeffs(L, 1, rng).astype(np.float32)
    lut = shm.bake_sh(torch.as_tensor(c).to(DEV), N)[0].cpu().numpy()
    t = sample_texels(N, 400, rng)
    got = lut[t[:, 0], t[:, 1], t[:, 2]]
    ref = np.array([oracle.bake_sh_point(c[0].astype(np.float64), N, int(f), (p - 0.5) / N, (q - 0.5) / N)
                    for f, q, p in t])
    check_lut(got, ref, f"L={L} N={N}")


def test_backward_largest_face():
    """N = 1,024, 2^20 directions: the LUT gradient through the adjoint
    identity, the direction gradient against the oracle on sampled queries."""
    N, Q = 1024, 1 << 20
    r = np.random.default_rng(11)
    dirs = workloads.uniform_dirs(Q, r)
    lut_np = workloads.random_lut(N, r)
    d_t, lut = torch.as_tensor(dirs).to(DEV), torch.as_tensor(lut_np).to(DEV)
    gen = torch.Generator(device=DEV).manual_seed(11)
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
    k = np.unique(np.concatenate([[0, Q - 1], r.choice(Q, 2000, replace=False)]))
    _, rd = oracle.backward(lut_np, dirs[k], g.cpu().numpy()[k], want_lut=False)
    gk = gd.cpu().numpy()[k]
    gn = np.linalg.norm(rd, axis=1)
    floor = np.sqrt(np.mean(gn ** 2))
    _e = np.linalg.norm(gk - rd, axis=1) / np.maximum(gn, floor)
    print('grad_dirs error max %.3e rms %.3e' % (_e.max(), np.sqrt(np.mean(_e ** 2))))
    assert _e.max() < 2e-5  # FP32 vs FP64 (measured <= 1e-6)


def test_trace_face_size_one():
    """A map with one cell per face: the ray cast against the oracle."""
    N = 1
    mu, amp, width = workloads.bump_params(workloads.rng_for(3))
    md = oracle.margin_dirs(N)
    samples = workloads.bumps_value(mu, amp, width, 1.0, md.reshape(-1, 3)).reshape(6, N + 4, N + 4)
    lut = oracle.bake_fd(samples, N).astype(np.float32)
    rmax = oracle.rmax_bound(lut.astype(np.float64)) * 1.0001
    o, d = workloads.camera_rays(48, 40)
    t, out, n = shm.trace(torch.as_tensor(lut).to(DEV), (0.0, 0.0, 0.0), rmax, torch.as_tensor(o).to(DEV),
                          torch.as_tensor(d).to(DEV), image_width=48)
    torch.cuda.synchronize()
    ref = oracle.trace(lut.astype(np.float64), np.zeros(3), rmax, o, d)
    assert np.isfinite(ref[0]).mean() > 0.2
    compare((t.cpu().numpy(), out.cpu().numpy(), n.cpu().numpy()), ref, "trace N=1", max_disagree=1.5 / o.shape[0])
    # bound maps with more blocks than cells: the same bits
    lg = torch.as_tensor(lut).to(DEV)
    for B in (1, 3, 64):
        b = shm.trace(lg, (0.0, 0.0, 0.0), rmax, torch.as_tensor(o).to(DEV), torch.as_tensor(d).to(DEV),
                      image_width=48, bound_map=shm.lut_bound_map(lg, blocks=B))
        for x, y in zip((t, out, n), b):
            assert torch.equal(x.view(torch.int32), y.view(torch.int32)), B
