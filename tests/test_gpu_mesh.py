"""Radial-depth bake from a triangle mesh (Sec. 4.9) on the GPU against the
FP64 oracle: ray cast of every direction against every triangle, then the
finite-difference bake of the samples."""
import numpy as np
import pytest
import torch

import oracle
import paper_2602_20063_amd as shm
import workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def gpu(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    return t.to(device=DEV, dtype=dtype) if dtype is not None else t.to(device=DEV)


def rel_err(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-30)


def test_mesh_depth_small_mesh_matches_oracle():
    """1,280 + 2 invalid triangles (ragged tile), 2,400 margin directions
    (ragged workgroup) plus zero and NaN directions."""
    prm = workloads.asteroid_params(np.random.default_rng(1))
    V, F = workloads.asteroid_mesh(prm, level=3)
    F = np.concatenate([F, [[0, 1, len(V)], [-5, 1, 2]]]).astype(np.int32)
    d = oracle.margin_dirs(18).reshape(-1, 3).astype(np.float32)
    d = np.concatenate([d, [[0, 0, 0], [np.nan, 1, 0]]]).astype(np.float32)
    c = (0.01, -0.02, 0.015)
    g = shm.mesh_radial_depth(gpu(V), gpu(F), c, gpu(d)).cpu().numpy()
    ref = oracle.mesh_radial_depth(V, F, np.array(c, np.float32), d)
    assert (g[-2:] == 0).all() and (ref[-2:] == 0).all()
    assert rel_err(g[:-2], ref[:-2]).max() < 2e-6


def test_mesh_depth_box_closed_form():
    a, c = np.float32(0.7), np.array([0.25, -1.5, 3.0], np.float32)
    lo, hi = c - a, c + a
    V = np.array([[hi[0] if i & 1 else lo[0], hi[1] if i & 2 else lo[1], hi[2] if i & 4 else lo[2]] for i in range(8)],
                 np.float32)
    quads = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    F = np.array([(q[0], q[1], q[2]) for q in quads] + [(q[0], q[2], q[3]) for q in quads], np.int32)
    d = workloads.uniform_dirs(50000, np.random.default_rng(2))
    g = shm.mesh_radial_depth(gpu(V), gpu(F), c, gpu(d)).cpu().numpy()
    w = d.astype(np.float64) / np.linalg.norm(d.astype(np.float64), axis=1, keepdims=True)
    assert rel_err(g, float(a) / np.abs(w).max(axis=1)).max() < 2e-6


def test_mesh_depth_asteroid_full_size_sampled():
    """The bench configuration: 81,920 triangles (40 triangle chunks combined
    by atomic max), the 6 x 52^2 margin grid of N = 48; the oracle checks a
    sample of the rays."""
    prm = workloads.asteroid_params(workloads.rng_for(6))
    V, F = workloads.asteroid_mesh(prm, level=6)
    N = 48
    d = shm.margin_dirs(N).reshape(-1, 3)
    g = shm.mesh_radial_depth(gpu(V), gpu(F), (0.0, 0.0, 0.0), d).cpu().numpy()
    dn = d.cpu().numpy()
    idx = np.random.default_rng(3).choice(dn.shape[0], 250, replace=False)
    ref = oracle.mesh_radial_depth(V, F, np.zeros(3), dn[idx])
    assert rel_err(g[idx], ref).max() < 2e-6
    assert (g > 0.7).all()
    # repeated calls give the same bits (the chunk maxima commute)
    g2 = shm.mesh_radial_depth(gpu(V), gpu(F), (0.0, 0.0, 0.0), d).cpu().numpy()
    assert np.array_equal(g, g2)


def test_bake_mesh_matches_oracle_chain():
    prm = workloads.asteroid_params(np.random.default_rng(4))
    V, F = workloads.asteroid_mesh(prm, level=3)
    N = 16
    lut = shm.bake_mesh(gpu(V), gpu(F), (0.0, 0.0, 0.0), N)[0].cpu().numpy()
    md = oracle.margin_dirs(N).reshape(-1, 3).astype(np.float32)
    ref = oracle.bake_fd(oracle.mesh_radial_depth(V, F, np.zeros(3), md).reshape(6, N + 4, N + 4), N)
    # FP32 depth samples (~1e-7 relative) enter every channel through sums
    # and differences of at most four samples
    assert np.abs(lut - ref).max() < 2e-6 * np.abs(ref[..., 0]).max()
