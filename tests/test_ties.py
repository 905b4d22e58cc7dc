"""The FP32/FP64 tie classifier (oracle.ties) on the CPU: keys decided by
the kernels' documented FP32 sequence (emulated here with numpy float32
operations, each correctly rounded) differ from the oracle's FP64 decision
only inside the tie band, and a planted non-tie difference is caught."""
import numpy as np

import oracle
import workloads
from oracle import ties

# face table of the hardware cube map (major axis M, sc axis S, tc axis T)
TM = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.float32)
TS = np.array([[0, 0, -1], [0, 0, 1], [1, 0, 0], [1, 0, 0], [1, 0, 0], [-1, 0, 0]], np.float32)
TT = np.array([[0, -1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1], [0, -1, 0], [0, -1, 0]], np.float32)


def fp32_keys(d, N):
    """The kernels' decision: a = sc/ma, u = (a+1)*0.5, f = u*N + 0.5,
    i0 = min(floor f, N), every step a correctly rounded float32 operation."""
    d = np.asarray(d, np.float32)
    ax, ay, az = np.abs(d).T
    face = np.where((ax >= ay) & (ax >= az), np.where(d[:, 0] >= 0, 0, 1),
                    np.where(ay >= az, np.where(d[:, 1] >= 0, 2, 3), np.where(d[:, 2] >= 0, 4, 5)))
    # products with +-1 / 0 and sums with one nonzero term: exact in float32
    ma = np.sum(d * TM[face], axis=1, dtype=np.float32)
    out = []
    for ax_tab in (TS, TT):
        sc = np.sum(d * ax_tab[face], axis=1, dtype=np.float32)
        a = (sc / ma).astype(np.float32)
        u = ((a + np.float32(1)).astype(np.float32) * np.float32(0.5)).astype(np.float32)
        f = ((u * np.float32(N)).astype(np.float32) + np.float32(0.5)).astype(np.float32)
        out.append(np.minimum(np.floor(f), N).astype(np.int64))
    i0, j0 = out
    C = N + 1
    return (face * C + j0) * C + i0


def test_fp32_sequence_differs_only_at_ties():
    d = workloads.uniform_dirs(2_000_000, np.random.default_rng(5))
    total = 0
    for N in (10, 32, 512, 1024):
        r = ties.classify(fp32_keys(d, N), d, N)
        assert r["ok"], (N, r)
        # the band is a few FP32 ulps of f wide, ~N ulp(1) at the face edges
        assert r["mismatches"] <= r["ties_in_band"] <= 1e-6 * N * r["queries"] + 10, (N, r)
        total += r["mismatches"]
    assert total > 0  # the emulated FP32 decision does pick neighbouring cells somewhere


def test_directions_placed_on_cell_edges_are_ties():
    """Directions built to land within an FP32 ulp of a cell edge: whatever
    cell the FP32 sequence picks, the classifier accepts it as a tie."""
    N = 64
    rng = np.random.default_rng(6)
    k = rng.integers(1, N + 1, 5000)
    u = (k - 0.5) / N + rng.uniform(-3e-7, 3e-7, k.size)
    v = rng.uniform(0.05, 0.95, k.size)
    d = np.stack([np.ones_like(u), -(2 * v - 1), -(2 * u - 1)], axis=1).astype(np.float32)  # +X face
    r = ties.classify(fp32_keys(d, N), d, N)
    assert r["ok"] and r["ties_in_band"] > 1000, r


def test_planted_non_tie_is_flagged():
    N = 32
    d = workloads.uniform_dirs(50000, np.random.default_rng(7))
    keys = fp32_keys(d, N)
    face, i0, j0, s, t = oracle.locate(d, N)
    mid = np.flatnonzero((s > 0.3) & (s < 0.7) & (i0 < N))[:3]
    bad = keys.copy()
    bad[mid] += 1  # the next cell along u, far from any edge
    r = ties.classify(bad, d, N)
    assert not r["ok"] and r["not_ties"] == 3, r
    bad = keys.copy()
    bad[mid[0]] += (N + 1) ** 2  # another face
    assert not ties.classify(bad, d, N)["ok"]
