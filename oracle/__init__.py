"""FP64 CPU oracle for Spherical Hermite Maps (arXiv 2602.20063).

TEST INFRASTRUCTURE ONLY.  The GPU library never imports or calls this
package; only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` do.  It shares no code with the HIP path: the arithmetic
lives in ``shm_oracle.c`` (plain C, IEEE double), this module only marshals
numpy arrays through ctypes.

Every function follows a passage of the paper:
  locate / query            Sec. 3.2 (cubemap face, padded grid), Sec. 3.3
                            Eqs. (3)-(5) (Hermite reconstruction, chart
                            derivatives), Sec. 3.4 Eqs. (6)-(10) (tangents,
                            metric tensor, Cramer solve, normal)
  bake_sh / bake_bumps      Sec. 3.3 Alg. 1, analytic SH derivatives via the
                            chain rule (computed with hyper-dual numbers)
  bake_fd / margin_dirs     Sec. 3.3 Alg. 1 general mode (central differences
                            with a bake-time margin)
  trace                     Sec. 3.1 (bounding sphere, bisection, Newton)
  backward                  gradients of the query outputs (exact adjoint of
                            the linear map LUT -> outputs; forward-mode in d)
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "shm_oracle.c")
_LIB = os.path.join(_HERE, "_shm_oracle.so")
# a sanitizer-instrumented build of the same source, loaded in place of the
# default one by the sanitizer test
_LIB_OVERRIDE = os.environ.get("SHM_ORACLE_LIB")

# -ffp-contract=off: no fused multiply-add anywhere, so the one FP32 decision
# (the ray caster's adaptive bisection budget) is the documented sequence of
# correctly rounded operations.
CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]


def build(force=False):
    """Compile shm_oracle.c into _shm_oracle.so with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            _lib = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB):
                build()
            _lib = ctypes.CDLL(_LIB)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def num_threads():
    """OpenMP threads the oracle runs with."""
    return int(lib().orc_num_threads())


def set_threads(n):
    """Number of OpenMP threads for the following oracle calls."""
    lib().orc_set_threads(ctypes.c_int(int(n)))


def lut_shape(N):
    return (6, N + 2, N + 2, 4)


def locate(dirs, N):
    """Face, cell (i0, j0) and local (s, t) per query (Sec. 3.2), all from
    the exact FP64 coordinate f = u N + 1/2 of the FP32 input: i0 =
    min(floor(f), N), s = f - i0 (likewise j0, t)."""
    d = _f32(dirs).reshape(-1, 3)
    Q = d.shape[0]
    face = np.empty(Q, np.int32)
    i0 = np.empty(Q, np.int32)
    j0 = np.empty(Q, np.int32)
    s = np.empty(Q)
    t = np.empty(Q)
    lib().orc_locate(_p(d), ctypes.c_int64(Q), ctypes.c_int(N), _p(face), _p(i0), _p(j0), _p(s), _p(t))
    return face, i0, j0, s, t


def query(lut, dirs, closed_form=False, normals=False):
    """(R, grad_x, grad_y, grad_z) per query [Q, 4] (+ normals [Q, 3])."""
    lut = _f64(lut)
    N = lut.shape[1] - 2
    assert lut.shape == lut_shape(N)
    d = _f32(dirs).reshape(-1, 3)
    Q = d.shape[0]
    out = np.empty((Q, 4))
    nrm = np.empty((Q, 3)) if normals else None
    lib().orc_query(_p(lut), ctypes.c_int(N), _p(d), ctypes.c_int64(Q), ctypes.c_int(1 if closed_form else 0), _p(out), _p(nrm))
    return (out, nrm) if normals else out


def query_f64(lut, dirs, face=-1):
    """FP64 directions with the cell decided in FP64; face >= 0 forces the
    face (both sides of a seam)."""
    lut = _f64(lut)
    N = lut.shape[1] - 2
    d = _f64(dirs).reshape(-1, 3)
    out = np.empty((d.shape[0], 4))
    lib().orc_query_f64(_p(lut), ctypes.c_int(N), _p(d), ctypes.c_int64(d.shape[0]), ctypes.c_int(face), _p(out))
    return out


def query_chart(lut, dirs):
    """Per query: r, r_u, r_v, det G, clamp flag, a=sc/ma, b=tc/ma, w (3)."""
    lut = _f64(lut)
    N = lut.shape[1] - 2
    d = _f32(dirs).reshape(-1, 3)
    Q = d.shape[0]
    out = np.empty((Q, 10))
    lib().orc_query_chart(_p(lut), ctypes.c_int(N), _p(d), ctypes.c_int64(Q), _p(out))
    return out


def reconstruct(lut, face, i0, j0, s, t):
    """(r, r_u, r_v) of cell (face, i0, j0) at local (s, t), Eqs. (4)-(5)."""
    lut = _f64(lut)
    N = lut.shape[1] - 2
    out = np.empty(3)
    lib().orc_reconstruct(_p(lut), ctypes.c_int(N), ctypes.c_int(face), ctypes.c_int(i0), ctypes.c_int(j0),
                          ctypes.c_double(s), ctypes.c_double(t), _p(out))
    return out


def query_objects(lut_flat, lut_off, Ns, q_begin, q_count, dirs, normals=False):
    """Batched queries over independent objects (flat FP64 LUT storage;
    lut_off in texels)."""
    lut_flat = _f64(lut_flat).reshape(-1)
    lut_off = np.ascontiguousarray(lut_off, np.int64)
    Ns = np.ascontiguousarray(Ns, np.int32)
    q_begin = np.ascontiguousarray(q_begin, np.int64)
    q_count = np.ascontiguousarray(q_count, np.int64)
    d = _f32(dirs).reshape(-1, 3)
    Q = d.shape[0]
    out = np.full((Q, 4), np.nan)
    nrm = np.full((Q, 3), np.nan) if normals else None
    lib().orc_query_objects(_p(lut_flat), _p(lut_off), _p(Ns), _p(q_begin), _p(q_count), ctypes.c_int64(len(Ns)),
                            _p(d), _p(out), _p(nrm))
    return (out, nrm) if normals else out


def hermite_basis(s):
    """(H0, H1, H0d, H1d, H0', H1', H0d', H1d') at s, Eq. (3)."""
    out = np.empty(8)
    lib().orc_hermite_basis(ctypes.c_double(s), _p(out))
    return out


def sh_basis(L, dirs):
    """Orthonormal real SH Y_k, k = l^2 + l + m, at unit directions."""
    d = _f64(dirs).reshape(-1, 3)
    K = (L + 1) ** 2
    Y = np.empty((d.shape[0], K))
    lib().orc_sh_basis(ctypes.c_int(L), _p(d), ctypes.c_int64(d.shape[0]), _p(Y))
    return Y


def sh_truth(coeffs, dirs):
    """Direct SH: (R, spherical gradient) at directions (need not be unit)."""
    c = _f64(coeffs).reshape(-1)
    L = int(round(np.sqrt(c.size))) - 1
    assert (L + 1) ** 2 == c.size
    d = _f64(dirs).reshape(-1, 3)
    out = np.empty((d.shape[0], 4))
    lib().orc_sh_truth(_p(c), ctypes.c_int(L), _p(d), ctypes.c_int64(d.shape[0]), _p(out))
    return out


def bake_sh(coeffs, N):
    """Alg. 1, analytic SH mode: FP64 LUT [6, N+2, N+2, 4] (or [n, ...] for a
    batch of coefficient vectors)."""
    c = _f64(coeffs)
    many = c.ndim == 2
    c2 = c.reshape(-1, c.shape[-1])
    L = int(round(np.sqrt(c2.shape[1]))) - 1
    assert (L + 1) ** 2 == c2.shape[1]
    lut = np.empty((c2.shape[0],) + lut_shape(N))
    lib().orc_bake_sh_many(_p(c2), ctypes.c_int(L), ctypes.c_int(N), ctypes.c_int64(c2.shape[0]), _p(lut))
    return lut if many else lut[0]


def bake_sh_point(coeffs, N, face, u, v):
    c = _f64(coeffs).reshape(-1)
    L = int(round(np.sqrt(c.size))) - 1
    out = np.empty(4)
    lib().orc_bake_sh_point(_p(c), ctypes.c_int(L), ctypes.c_int(N), ctypes.c_int(face), ctypes.c_double(u),
                            ctypes.c_double(v), _p(out))
    return out


def bake_bumps(mu, amp, width, base, N):
    mu = _f64(mu).reshape(-1, 3)
    amp = _f64(amp).reshape(-1)
    width = _f64(width).reshape(-1)
    lut = np.empty(lut_shape(N))
    lib().orc_bake_bumps(_p(mu), _p(amp), _p(width), ctypes.c_int(len(amp)), ctypes.c_double(base), ctypes.c_int(N), _p(lut))
    return lut


def bumps_truth(mu, amp, width, base, dirs):
    mu = _f64(mu).reshape(-1, 3)
    amp = _f64(amp).reshape(-1)
    width = _f64(width).reshape(-1)
    d = _f64(dirs).reshape(-1, 3)
    out = np.empty((d.shape[0], 4))
    lib().orc_bumps_truth(_p(mu), _p(amp), _p(width), ctypes.c_int(len(amp)), ctypes.c_double(base), _p(d),
                          ctypes.c_int64(d.shape[0]), _p(out))
    return out


def margin_dirs(N):
    """Unit directions of the padded grid plus a one-texel margin,
    [6, N+4, N+4, 3]."""
    out = np.empty((6, N + 4, N + 4, 3))
    lib().orc_margin_dirs(ctypes.c_int(N), _p(out))
    return out


def bake_fd(samples, N):
    """Alg. 1 general mode: central differences of samples [6, N+4, N+4]."""
    s = _f64(samples).reshape(6, N + 4, N + 4)
    lut = np.empty(lut_shape(N))
    lib().orc_bake_fd(_p(s), ctypes.c_int(N), _p(lut))
    return lut


def backward(lut, dirs, grad_out, want_lut=True, want_dirs=True):
    """Gradients of L = sum_q grad_out[q] . (R, grad R)(q) with respect to the
    LUT (FP64, LUT shape) and to the directions [Q, 3]."""
    lut = _f64(lut)
    N = lut.shape[1] - 2
    d = _f32(dirs).reshape(-1, 3)
    Q = d.shape[0]
    g = _f64(grad_out).reshape(Q, 4)
    gl = np.empty(lut_shape(N)) if want_lut else None
    gd = np.empty((Q, 3)) if want_dirs else None
    lib().orc_backward(_p(lut), ctypes.c_int(N), _p(d), ctypes.c_int64(Q), _p(g), _p(gl), _p(gd))
    return gl, gd


def rmax_bound(lut, absval=False):
    """Bernstein (convex hull) upper bound of the reconstruction over all
    cells (of its absolute value with absval, for signed functions)."""
    lut = _f64(lut)
    N = lut.shape[1] - 2
    lib().orc_rmax_bound.restype = ctypes.c_double
    return float(lib().orc_rmax_bound(_p(lut), ctypes.c_int(N), ctypes.c_int(1 if absval else 0)))


def cell_bezier(lut, face, i0, j0):
    """Bezier control net [4 (s), 4 (t)] of one cell's bicubic patch."""
    lut = _f64(lut)
    N = lut.shape[1] - 2
    out = np.empty((4, 4))
    lib().orc_cell_bezier(_p(lut), ctypes.c_int(N), ctypes.c_int(face), ctypes.c_int(i0), ctypes.c_int(j0), _p(out))
    return out


def trace(lut, center, rmax, ray_o, ray_d, n_march=20, n_bisect=8, n_newton=3):
    """Sec. 3.1 ray casting: t [P] (+inf = miss), (R, grad) [P, 4], normal [P, 3]."""
    lut = _f64(lut)
    N = lut.shape[1] - 2
    o = _f32(ray_o).reshape(-1, 3)
    d = _f32(ray_d).reshape(-1, 3)
    P = o.shape[0]
    c = _f64(center).reshape(3)
    t = np.empty(P)
    out = np.empty((P, 4))
    nrm = np.empty((P, 3))
    lib().orc_trace(_p(lut), ctypes.c_int(N), _p(c), ctypes.c_double(rmax), _p(o), _p(d), ctypes.c_int64(P),
                    ctypes.c_int(n_march), ctypes.c_int(n_bisect), ctypes.c_int(n_newton), _p(t), _p(out), _p(nrm))
    return t, out, nrm


def trace_ex(lut, center, rmax, ray_o, ray_d, scale=1.0, signed=False, px=0.0, eps_px=0.125, n_march=20,
             n_bisect=16, n_newton=3):
    """Ray casting of the rendered radius R = scale r (scale |r| if signed)
    with the adaptive bisection budget (px = focal length in pixels; 0 for
    the fixed count n_bisect).  rmax bounds R; centre and rmax are taken as
    FP32.  Returns t, (R, grad) [P, 4], normal [P, 3], sign of r [P] int8,
    F evaluations [P] int32."""
    lut = _f64(lut)
    N = lut.shape[1] - 2
    o = _f32(ray_o).reshape(-1, 3)
    d = _f32(ray_d).reshape(-1, 3)
    P = o.shape[0]
    c = _f32(center).reshape(3)
    t = np.empty(P)
    out = np.empty((P, 4))
    nrm = np.empty((P, 3))
    sgn = np.empty(P, dtype=np.int8)
    ev = np.empty(P, dtype=np.int32)
    lib().orc_trace_ex(_p(lut), ctypes.c_int(N), _p(c), ctypes.c_float(rmax), ctypes.c_double(scale),
                       ctypes.c_int(1 if signed else 0), ctypes.c_float(px), ctypes.c_float(eps_px), _p(o), _p(d),
                       ctypes.c_int64(P), ctypes.c_int(n_march), ctypes.c_int(n_bisect), ctypes.c_int(n_newton), _p(t),
                       _p(out), _p(nrm), _p(sgn), _p(ev))
    return t, out, nrm, sgn, ev


def bisect_budget(o, center, rmax, px, eps_px, n_march, n_bisect):
    """The trace's per-ray bisection count (FP32 decision)."""
    o = _f32(o).reshape(3)
    c = _f32(center).reshape(3)
    return int(lib().orc_bisect_budget(_p(o), _p(c), ctypes.c_float(rmax), ctypes.c_float(px), ctypes.c_float(eps_px),
                                       ctypes.c_int(n_march), ctypes.c_int(n_bisect)))


def query_scaled(lut, dirs, scale=1.0, signed=False):
    """Rendered radius R = scale r (scale |r| if signed, gradient
    scale sign(r) grad r): (R, grad) [Q, 4], normal [Q, 3], sign [Q] int8."""
    lut = _f64(lut)
    N = lut.shape[1] - 2
    d = _f32(dirs).reshape(-1, 3)
    Q = d.shape[0]
    out = np.empty((Q, 4))
    nrm = np.empty((Q, 3))
    sgn = np.empty(Q, dtype=np.int8)
    lib().orc_query_scaled(_p(lut), ctypes.c_int(N), _p(d), ctypes.c_int64(Q), ctypes.c_double(scale),
                           ctypes.c_int(1 if signed else 0), _p(out), _p(nrm), _p(sgn))
    return out, nrm, sgn


def trace_F(lut, center, o, d, ts):
    lut = _f64(lut)
    N = lut.shape[1] - 2
    ts = _f64(ts).reshape(-1)
    F = np.empty(ts.size)
    lib().orc_trace_F(_p(lut), ctypes.c_int(N), _p(_f64(center)), _p(_f64(o)), _p(_f64(d)), _p(ts),
                      ctypes.c_int64(ts.size), _p(F))
    return F


BASELINE_NEAREST, BASELINE_BILINEAR_FD, BASELINE_BICUBIC, BASELINE_FAST_BICUBIC_FD = 0, 1, 2, 3


def baseline_query(vlut, dirs, method):
    """Comparison reconstructions on a value-only LUT [6, N+4, N+4] (texel p
    at u = (p - 3/2)/N): 0 nearest, 1 bilinear + finite-difference
    gradient, 2 Catmull-Rom bicubic + analytic gradient, 3 cubic B-spline
    ("fast bicubic") + the finite-difference gradient of 1.  (R, grad) [Q, 4]."""
    v = _f64(vlut)
    N = v.shape[-1] - 4
    d = _f32(dirs).reshape(-1, 3)
    out = np.empty((d.shape[0], 4))
    lib().orc_baseline_query(_p(v), ctypes.c_int(N), _p(d), ctypes.c_int64(d.shape[0]), ctypes.c_int(method), _p(out))
    return out


def mip_level(lut, naive=False):
    """Next mip level (N -> N/2) of a TEXEL LUT: derivative-consistent
    (filtered values, derivatives by central differences) or naive (box
    filter of all four stored channels of interior texels)."""
    lut = _f64(lut)
    N = lut.shape[1] - 2
    assert N % 2 == 0
    out = np.empty(lut_shape(N // 2))
    lib().orc_mip_level(_p(lut), ctypes.c_int(N), ctypes.c_int(1 if naive else 0), _p(out))
    return out


def mesh_radial_depth(verts, tris, center, dirs):
    """R(w) = max{t >= 0 : c + t w on the mesh} per direction (0 if none),
    by testing every triangle in FP64.  verts [V, 3], tris [T, 3] int."""
    v = _f64(verts).reshape(-1, 3)
    t = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    c = _f64(center).reshape(3)
    d = _f32(dirs).reshape(-1, 3)
    out = np.empty(d.shape[0])
    lib().orc_mesh_radial_depth(_p(v), ctypes.c_int64(v.shape[0]), _p(t), ctypes.c_int64(t.shape[0]), _p(c), _p(d),
                                ctypes.c_int64(d.shape[0]), _p(out))
    return out
