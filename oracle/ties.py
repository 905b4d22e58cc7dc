"""FP32 / FP64 cell-decision ties (Sec. 3.2: the query's cell is the floor
of the continuous padded coordinate f = u N + 1/2).

Test infrastructure, like the rest of this package: only the tests, the
smoke check and the benchmark's CPU leg use it.

The oracle takes the decision on the exact FP64 coordinate.  The kernels take
it in FP32 by a documented sequence (a = sc/ma, u = (a + 1) * 0.5,
f = u * N + 0.5, i0 = min(floor f, N), each step correctly rounded), whose
result differs from the exact f by at most

    |f32 - f| <= (N/4) ulp(a) + (N/2) ulp(u) + ulp(f)

(half an ulp per rounding, carried through the scalings).  A query is a
*tie* when its FP64 coordinate lies within twice that bound of an integer
(a cell edge): there the two precisions may pick neighbouring cells, and
the value and gradient still agree because the Hermite patch is C1 across
cell edges.  Faces are decided by comparisons that are exact in any
precision, so they must always agree.
"""
import numpy as np

from . import locate


def _ulp32(x):
    x = np.abs(np.asarray(x, np.float64)).astype(np.float32)
    return np.spacing(x).astype(np.float64)


def tie_band(f, N):
    """Twice the FP32 sequence's error bound on f, per coordinate."""
    f = np.asarray(f, np.float64)
    u = (f - 0.5) / N
    a = 2.0 * u - 1.0
    return 2.0 * ((N / 4.0) * _ulp32(a) + (N / 2.0) * _ulp32(u) + _ulp32(f))


def fp64_keys(dirs, N, q_per_obj=None):
    """Cell keys ((obj * 6 + face) * (N+1) + j0) * (N+1) + i0 of the oracle's
    FP64 decision (0xFFFFFFFF for invalid directions) and the FP64
    coordinates (fu, fv)."""
    d = np.asarray(dirs, np.float32).reshape(-1, 3)
    Q = d.shape[0]
    face, i0, j0, s, t = locate(d, N)
    obj = np.zeros(Q, np.int64) if q_per_obj is None else np.arange(Q, dtype=np.int64) // q_per_obj
    C = N + 1
    keys = (((obj * 6 + face) * C + j0) * C + i0).astype(np.int64)
    keys[face < 0] = 0xFFFFFFFF
    return keys, face, i0 + s, j0 + t


def classify(gpu_keys, dirs, N, q_per_obj=None):
    """Compare the kernels' cell keys with the FP64 decision.

    Returns a dict: mismatches (count), ties_in_band (FP64 coordinates within
    the tie band of a cell edge, whatever was decided), and 'ok' = every
    mismatch is a tie (same object and face, a neighbouring cell, and the
    coordinate of each differing axis inside the band).  Faces and invalid
    directions must agree exactly."""
    g = np.asarray(gpu_keys).astype(np.int64) & 0xFFFFFFFF
    k64, face, fu, fv = fp64_keys(dirs, N, q_per_obj)
    assert g.shape == k64.shape
    valid = face >= 0
    assert np.array_equal(g == 0xFFFFFFFF, ~valid), "invalid directions differ"
    C = N + 1
    gi, gj = g % C, (g // C) % C
    gfo = g // (C * C)
    ei, ej = k64 % C, (k64 // C) % C
    efo = k64 // (C * C)
    bu, bv = tie_band(fu, N), tie_band(fv, N)
    near_u = np.abs(fu - np.round(fu)) <= bu
    near_v = np.abs(fv - np.round(fv)) <= bv
    mis = valid & (g != k64)
    di, dj = np.abs(gi - ei), np.abs(gj - ej)
    tie_ok = (gfo == efo) & (di <= 1) & (dj <= 1) & ((di == 0) | near_u) & ((dj == 0) | near_v)
    bad = mis & ~tie_ok
    return {"mismatches": int(mis.sum()), "ties_in_band": int((valid & (near_u | near_v)).sum()),
            "not_ties": int(bad.sum()), "ok": not bad.any(), "bad_index": np.flatnonzero(bad)[:10].tolist(),
            "queries": int(valid.sum())}
