"""The seeded generators: reproducibility, distributions and the two
implementations of the fBm target."""
import math

import numpy as np
import torch

import workloads


def test_seeded_and_unit():
    a = workloads.uniform_dirs(1000, workloads.rng_for(2))
    b = workloads.uniform_dirs(1000, workloads.rng_for(2))
    assert np.array_equal(a, b) and a.dtype == np.float32
    assert np.abs(np.linalg.norm(a.astype(np.float64), axis=1) - 1).max() < 1e-6


def test_glyph_radius_range():
    """R = 1 + 0.3 SH / B with B >= max |SH| keeps R inside [0.7, 1.3]."""
    import oracle

    c = workloads.sh_glyph_coeffs(8, 4, workloads.rng_for(2))
    assert c.shape == (4, 81)
    d = workloads.uniform_dirs(20000, np.random.default_rng(3)).astype(np.float64)
    for k in range(4):
        R = oracle.sh_truth(c[k], d)[:, 0]
        assert 0.7 <= R.min() and R.max() <= 1.3
        assert R.max() - R.min() > 0.05


def test_fbm_numpy_and_torch_agree_and_gradient():
    d = workloads.uniform_dirs(3000, np.random.default_rng(1)).astype(np.float64)
    v, g = workloads.fbm_target(d, 7)
    vt, gt = workloads.fbm_target_torch(torch.as_tensor(d), 7)
    assert np.abs(v - vt.numpy()).max() < 1e-12
    assert np.abs(g - gt.numpy()).max() < 1e-9
    assert 0.7 < v.min() and v.max() < 1.3
    # gradient vs central differences along a tangent direction
    w = d / np.linalg.norm(d, axis=1, keepdims=True)
    tau = np.cross(w, np.array([0.3, 0.5, 0.8]))
    tau /= np.linalg.norm(tau, axis=1, keepdims=True)
    h = 1e-6
    fp, _ = workloads.fbm_target(w + h * tau, 7)
    fm, _ = workloads.fbm_target(w - h * tau, 7)
    fd = (fp - fm) / (2 * h)
    assert np.abs(fd - np.sum(g * tau, axis=1)).max() < 1e-5


def test_uneven_batch_distribution():
    spec = workloads.uneven_batch(workloads.rng_for(5))
    assert len(spec["N"]) == 4096
    assert set(np.unique(spec["N"])) <= set(workloads.BATCH_NS)
    assert spec["Q"].min() >= 64 and spec["Q"].max() <= 1 << 20
    assert 2 <= spec["L"].min() and spec["L"].max() <= 16
    assert 6e7 < spec["Q"].sum() < 1.6e8
