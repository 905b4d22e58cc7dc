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


def test_real_sh_convention_matches_the_oracle():
    """The generator's real SH (scipy's complex harmonics, phase removed) is
    the convention the oracle bakes in: orthonormal, no Condon-Shortley
    phase, k = l^2 + l + m (Y_1,1 ~ +x, Y_1,-1 ~ +y)."""
    import oracle

    d = workloads.uniform_dirs(2000, np.random.default_rng(5)).astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    for L in (2, 8, 16):
        Y = workloads.real_sh(L, d)
        scale = np.abs(Y).max()
        assert np.abs(Y - oracle.sh_basis(L, d)).max() < 1e-12 * scale, L
    k = math.sqrt(3.0 / (4.0 * math.pi))
    Y1 = workloads.real_sh(1, d)
    np.testing.assert_allclose(Y1[:, 1:], k * d[:, [1, 2, 0]], atol=1e-14)


def test_fibonacci_sphere():
    p = workloads.fibonacci_sphere(4096)
    assert p.shape == (4096, 3)
    assert np.abs(np.linalg.norm(p, axis=1) - 1).max() < 1e-14
    assert np.abs(p.mean(axis=0)).max() < 1e-3  # spread evenly
    # nearest-neighbour spacing close to the equal-area spacing sqrt(4 pi / n)
    sub = p[::64]
    dmin = np.sort(np.linalg.norm(sub[:, None] - p[None], axis=2), axis=1)[:, 1]
    assert 0.6 * math.sqrt(4 * math.pi / 4096) < dmin.min() and dmin.max() < 1.6 * math.sqrt(4 * math.pi / 4096)


def test_glyph_radius_range():
    """R = 1 + 0.3 SH / max|SH| with the maximum over the 4,096-point
    Fibonacci sphere: |R - 1| reaches exactly 0.3 there, and stays within a
    few percent of it anywhere else on the sphere."""
    import oracle

    c = workloads.sh_glyph_coeffs(8, 4, workloads.rng_for(2))
    assert c.shape == (4, 81)
    fib = workloads.fibonacci_sphere(4096)
    d = workloads.uniform_dirs(20000, np.random.default_rng(3)).astype(np.float64)
    for k in range(4):
        Rf = oracle.sh_truth(c[k], fib)[:, 0]
        assert abs(np.abs(Rf - 1).max() - 0.3) < 1e-12
        assert 0.7 - 1e-12 <= Rf.min() and Rf.max() <= 1.3 + 1e-12
        R = oracle.sh_truth(c[k], d)[:, 0]
        assert np.abs(R - 1).max() < 0.3 * 1.05
        assert R.max() - R.min() > 0.2


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
