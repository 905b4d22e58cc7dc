"""Tolerance rules for comparing the HIP path with the FP64 oracle.

FP32 arithmetic against the FP64 oracle on the same LUT data:
  value     |dR| <= 1e-5 |R_ref|
  gradient  |d grad| <= 1e-4 max(|grad_ref|, RMS over the batch of |grad_ref|)
(the second floor keeps the relative test meaningful where the gradient
vanishes).  Integer decisions (face, cell) must be bit-identical.
"""
import numpy as np

VAL_RTOL = 1e-5
GRAD_RTOL = 1e-4


def check_value_grad(out, ref, what="", val_rtol=VAL_RTOL, grad_rtol=GRAD_RTOL):
    out = np.asarray(out, np.float64)
    ref = np.asarray(ref, np.float64)
    assert out.shape == ref.shape
    nan_o = np.isnan(out[:, 0])
    nan_r = np.isnan(ref[:, 0])
    assert np.array_equal(nan_o, nan_r), f"{what}: NaN pattern differs ({nan_o.sum()} vs {nan_r.sum()})"
    ok = ~nan_r
    o, r = out[ok], ref[ok]
    if o.shape[0] == 0:
        return {"n": 0}
    dv = np.abs(o[:, 0] - r[:, 0]) / np.maximum(np.abs(r[:, 0]), 1e-30)
    gn = np.linalg.norm(r[:, 1:], axis=1)
    floor = np.sqrt(np.mean(gn ** 2))
    dg = np.linalg.norm(o[:, 1:] - r[:, 1:], axis=1) / np.maximum(np.maximum(gn, floor), 1e-30)
    stats = {"n": int(o.shape[0]), "val_max_rel": float(dv.max()), "grad_max_rel": float(dg.max()),
             "val_rms_rel": float(np.sqrt(np.mean(dv ** 2))), "grad_rms_rel": float(np.sqrt(np.mean(dg ** 2)))}
    assert dv.max() <= val_rtol, f"{what}: value error {dv.max():.3e} > {val_rtol} at {np.argmax(dv)}"
    assert dg.max() <= grad_rtol, f"{what}: gradient error {dg.max():.3e} > {grad_rtol} at {np.argmax(dg)}"
    return stats


def angle_deg(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    c = np.sum(a * b, axis=1) / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1))
    return np.degrees(np.arccos(np.clip(c, -1.0, 1.0)))


def decode_f16_cells(c16):
    """FP16 cells (the library's FP16 cell encoding: corners 1..3 hold r as a
    difference from corner 0's r) -> the FP32 footprints a query decodes
    (one FP32 addition per corner), same shape."""
    c = np.asarray(c16).astype(np.float32).reshape(-1, 4, 4).copy()
    c[:, 1:, 0] += c[:, :1, 0]
    return c.reshape(np.asarray(c16).shape)
