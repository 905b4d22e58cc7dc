"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/shm.h, and rejects bad arguments with
the documented status codes before anything is enqueued."""
import ctypes
import glob
import os
import re

import pytest

import paper_2602_20063_amd as shm
from conftest import ROOT

HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_symbols():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^SHM_API\s+[\w\s\*]+?\b(shm_\w+)\(", text, flags=re.M)))


def test_library_loads_and_exports_every_declared_symbol():
    L = shm.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
        assert n in shm.SIGNATURES, f"{n} has no Python binding"
    assert set(shm.SIGNATURES) == set(names)


def test_version_and_sizes():
    assert shm.shm_version() == 1
    assert shm.shm_lut_elems(10, shm.SHM_LAYOUT_TEXEL) == 6 * 12 * 12 * 4
    assert shm.shm_lut_elems(32, shm.SHM_LAYOUT_CELL) == 6 * 33 * 33 * 16
    assert shm.shm_lut_elems(0, 0) == 0
    assert shm.shm_lut_elems(2000, 0) == 0
    assert shm.shm_lut_elems(4, 7) == 0
    # basis table: padded K x padded rows, FP32
    assert shm.shm_bake_sh_lut_workspace(8, 32) >= 81 * 6 * 34 * 34 * 4 * 4
    assert shm.shm_bake_sh_lut_workspace(17, 32) == 0
    # two (key, index) buffers of 8 B per query, cell starts, digit histograms
    ws = shm.shm_backward_workspace(512, 1, 1 << 22)
    assert (1 << 22) * 16 + 6 * 513 * 513 * 4 <= ws < (1 << 22) * 20


def call(name, *args):
    return getattr(shm.lib(), name)(*args)


def test_query_argument_validation():
    """Each bad argument gives its status code and a message naming it; an
    accepted call clears the message."""
    p = ctypes.c_void_p(16)
    cases = [
        ((p, 5, 0, 10, 1, p, 8, p, None, None), shm.SHM_ERR_INVALID_ARG, "bad dtype"),
        ((p, 0, 3, 10, 1, p, 8, p, None, None), shm.SHM_ERR_INVALID_ARG, "bad layout"),
        ((p, 0, 0, 0, 1, p, 8, p, None, None), shm.SHM_ERR_INVALID_ARG, "N must be"),
        ((p, 0, 0, 1025, 1, p, 8, p, None, None), shm.SHM_ERR_INVALID_ARG, "N must be"),
        ((p, 0, 0, 10, -1, p, 8, p, None, None), shm.SHM_ERR_INVALID_ARG, "negative size"),
        ((None, 0, 0, 10, 1, p, 8, p, None, None), shm.SHM_ERR_INVALID_ARG, "null pointer"),
        ((p, 0, 0, 10, 1, p, 8, ctypes.c_void_p(20), None, None), shm.SHM_ERR_INVALID_ARG, "misaligned"),
        ((p, 0, 0, 10, 0, p, 8, p, None, None), shm.SHM_OK, ""),  # empty: nothing to do
        ((p, 0, 0, 10, 3, p, 0, p, None, None), shm.SHM_OK, ""),
    ]
    for args, code, msg in cases:
        assert call("shm_query_value_grad", *args) == code, args
        err = shm.shm_last_error()
        if code == shm.SHM_OK:
            assert err == "", (args, err)
        else:
            assert msg in err, (args, err)


def test_error_message_is_set():
    p = ctypes.c_void_p(16)
    assert call("shm_query_value_grad", p, 0, 0, 0, 1, p, 8, p, None, None) == shm.SHM_ERR_INVALID_ARG
    assert "N must be" in shm.shm_last_error()


def test_bake_argument_validation():
    p = ctypes.c_void_p(256)
    assert call("shm_bake_sh_lut", p, 17, 8, 1, 0, p, p, 1 << 30, None) == shm.SHM_ERR_UNSUPPORTED
    assert call("shm_bake_sh_lut", p, -1, 8, 1, 0, p, p, 1 << 30, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_bake_sh_lut", p, 4, 8, 1, 0, p, p, 16, None) == shm.SHM_ERR_WORKSPACE
    assert call("shm_bake_sh_lut", p, 4, 8, 1, 0, p, None, 1 << 30, None) == shm.SHM_ERR_WORKSPACE
    assert call("shm_bake_sh_lut", p, 4, 8, 1, 9, p, p, 1 << 30, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_bake_sh_lut", p, 4, 8, 0, 0, None, None, 0, None) == shm.SHM_OK


def test_backward_and_trace_validation():
    p = ctypes.c_void_p(256)
    assert call("shm_backward_sort", 8, 1, p, 100, p, 10, None) == shm.SHM_ERR_WORKSPACE
    assert call("shm_backward_sort", 0, 1, p, 100, p, 1 << 30, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_backward_sort", 8, 1, p, 100, ctypes.c_void_p(300), 1 << 30, None) == shm.SHM_ERR_INVALID_ARG
    # sort_ready takes 0, SHM_SORT_READY or SHM_SORT_READY_SPARSE only
    qb = lambda sr: call("shm_query_backward", p, 8, 1, p, 100, p, p, p, p, 1 << 30, sr, None)
    for sr in (-1, 3):
        assert qb(sr) == shm.SHM_ERR_INVALID_ARG
        assert "sort_ready" in shm.lib().shm_last_error().decode()
    # the dense-tile count: nothing to read without queries, -1 for bad arguments
    dt = lambda *a: shm.lib().shm_backward_dense_tiles(*a)
    assert dt(8, 1, 0, p, 1 << 30, None) == 0
    assert dt(8, 0, 100, p, 1 << 30, None) == 0
    assert dt(0, 1, 100, p, 1 << 30, None) == -1
    assert dt(8, 1, 100, p, 10, None) == -1
    assert dt(8, 1, 100, ctypes.c_void_p(300), 1 << 30, None) == -1
    assert "workspace" in shm.lib().shm_last_error().decode()
    c = (ctypes.c_float * 3)(0, 0, 0)
    assert call("shm_trace_radial", p, 0, 8, c, ctypes.c_float(-1.0), p, p, 10, 20, 8, 3, p, p, None, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_trace_radial", p, 0, 8, c, ctypes.c_float(1.0), p, p, 10, 40, 20, 10, p, p, None, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_trace_radial", p, 0, 8, None, ctypes.c_float(1.0), p, p, 10, 20, 8, 3, p, p, None, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_trace_radial", p, 0, 8, c, ctypes.c_float(1.0), p, p, 0, 20, 8, 3, p, p, None, None) == shm.SHM_OK


def test_plan_validation():
    h = ctypes.c_void_p()
    objs = (shm.shm_object * 2)()
    objs[0].lut_offset, objs[0].N, objs[0].q_begin, objs[0].q_count = 0, 8, 0, 10
    objs[1].lut_offset, objs[1].N, objs[1].q_begin, objs[1].q_count = 3, 8, 10, 10  # misaligned offset
    assert call("shm_plan_create", ctypes.cast(objs, ctypes.c_void_p), 2, 0, 0, None, ctypes.byref(h)) == shm.SHM_ERR_INVALID_ARG
    objs[1].lut_offset, objs[1].N = 4, 0
    assert call("shm_plan_create", ctypes.cast(objs, ctypes.c_void_p), 2, 0, 0, None, ctypes.byref(h)) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_plan_create", None, 2, 0, 0, None, ctypes.byref(h)) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_plan_launch", None, None, None, None, None, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_plan_graph_launch", None, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_plan_destroy", None) == shm.SHM_OK
    assert shm.lib().shm_plan_work_items(None) == -1
    s = shm.shm_launch_shape(100, 1, 100, 4)
    assert call("shm_plan_set_shape", None, ctypes.byref(s)) == shm.SHM_ERR_INVALID_ARG


def test_render_validation():
    """Rendered-radius query and trace: scale, flags and budget parameters
    are checked on the host before anything is enqueued."""
    p = ctypes.c_void_p(256)
    c = (ctypes.c_float * 3)(0, 0, 0)

    def prm(**kw):
        d = dict(scale=1.0, flags=0, n_march=20, n_bisect=8, n_newton=3, px_per_unit=0.0, eps_px=0.0, image_width=0,
                 bound_blocks=0, bound_map=None)
        d.update(kw)
        return shm.shm_trace_params(**d)

    def tr(pp, P=10):
        return call("shm_trace_radial_ex", p, 0, 8, c, 1.0, ctypes.byref(pp), p, p, P, p, p, None, None, None, None)

    assert tr(prm(), P=0) == shm.SHM_OK
    assert tr(prm(flags=shm.SHM_SIGNED, px_per_unit=900.0, eps_px=0.1), P=0) == shm.SHM_OK
    for bad in (prm(scale=0.0), prm(scale=float("inf")), prm(flags=4), prm(n_march=0), prm(n_bisect=60),
                prm(px_per_unit=-1.0), prm(px_per_unit=float("nan")), prm(px_per_unit=100.0, eps_px=0.0),
                prm(image_width=-1), prm(image_width=3), prm(image_width=20),
                prm(bound_blocks=-1), prm(bound_blocks=65, bound_map=256), prm(bound_blocks=4)):
        assert tr(bad) == shm.SHM_ERR_INVALID_ARG  # 10 rays: not whole rows of 3 or 20; map sizes
    assert tr(prm(image_width=7), P=0) == shm.SHM_OK
    # cell LUTs are read with 16-byte loads, FP16 ones included
    p8 = ctypes.c_void_p(264)
    assert call("shm_trace_radial_ex", p8, 1, 8, c, 1.0, ctypes.byref(prm(flags=shm.SHM_CELL_LUT)), p, p, 10, p, p,
                None, None, None, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_lut_rmax", p8, 1, 8, shm.SHM_CELL_LUT, p, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_lut_bound_map", p8, 1, 8, shm.SHM_CELL_LUT, 4, p, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_lut_rmax", p, 0, 8, 4, p, None) == shm.SHM_ERR_INVALID_ARG  # unknown flag
    assert call("shm_trace_radial_ex", p, 0, 8, c, 1.0, None, p, p, 10, p, p, None, None, None, None) == shm.SHM_ERR_INVALID_ARG
    q = lambda scale, flags, Q=10: call("shm_query_scaled", p, 0, 0, 8, 1, p, Q, scale, flags, p, None, None, None)
    assert q(0.0, 0) == shm.SHM_ERR_INVALID_ARG
    assert q(float("nan"), 0) == shm.SHM_ERR_INVALID_ARG
    assert q(1.0, 4) == shm.SHM_ERR_INVALID_ARG
    assert q(1.0, shm.SHM_SIGNED, Q=0) == shm.SHM_OK
    assert call("shm_query_scaled", p, 0, 0, 8, 1, None, 10, 1.0, 0, p, None, None, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_lut_rmax", p, 0, 8, 4, p, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_lut_rmax", p, 0, 8, 0, None, None) == shm.SHM_ERR_INVALID_ARG
    bm = lambda *a: call("shm_lut_bound_map", *a)
    for args in ((p, 0, 8, 0, 0, p), (p, 0, 8, 0, 65, p), (p, 0, 8, 4, 8, p), (None, 0, 8, 0, 8, p), (p, 0, 8, 0, 8, None),
                 (p, 0, 0, 0, 8, p), (p, 5, 8, 0, 8, p), (p, 0, 8, 0, 8, ctypes.c_void_p(258))):
        assert bm(*args, None) == shm.SHM_ERR_INVALID_ARG, args


def test_mesh_depth_validation():
    p = ctypes.c_void_p(256)
    c = (ctypes.c_float * 3)(0, 0, 0)
    cbad = (ctypes.c_float * 3)(0, float("nan"), 0)
    f = lambda *a: call("shm_mesh_radial_depth", *a)
    assert f(p, 8, p, 12, c, p, 0, p, None) == shm.SHM_OK          # no rays: nothing to do
    assert f(p, -1, p, 12, c, p, 10, p, None) == shm.SHM_ERR_INVALID_ARG
    assert f(p, 8, p, 12, None, p, 10, p, None) == shm.SHM_ERR_INVALID_ARG
    assert f(p, 8, p, 12, cbad, p, 10, p, None) == shm.SHM_ERR_INVALID_ARG
    assert f(p, 8, None, 12, c, p, 10, p, None) == shm.SHM_ERR_INVALID_ARG
    assert f(p, 8, p, 12, c, None, 10, p, None) == shm.SHM_ERR_INVALID_ARG
    assert f(p, 1 << 32, p, 12, c, p, 10, p, None) == shm.SHM_ERR_UNSUPPORTED
    assert f(p, 8, p, 12, c, p, 10, ctypes.c_void_p(258), None) == shm.SHM_ERR_INVALID_ARG


def test_fit_validation():
    """Loss gradient and Adam update: sizes, pointers, alignment and
    hyper-parameters are checked on the host before anything is enqueued."""
    p = ctypes.c_void_p(256)
    mis = ctypes.c_void_p(260)
    lg = lambda *a: call("shm_fit_loss_grad", *a)
    assert lg(p, p, p, p, 0, 1.0, p, None) == shm.SHM_OK
    assert lg(p, p, p, p, -1, 1.0, p, None) == shm.SHM_ERR_INVALID_ARG
    assert lg(p, p, p, p, 10, float("nan"), p, None) == shm.SHM_ERR_INVALID_ARG
    assert lg(p, p, p, p, 10, -1.0, p, None) == shm.SHM_ERR_INVALID_ARG
    assert lg(None, p, p, p, 10, 1.0, p, None) == shm.SHM_ERR_INVALID_ARG
    assert lg(p, p, p, p, 10, 1.0, None, None) == shm.SHM_ERR_INVALID_ARG
    assert lg(mis, p, p, p, 10, 1.0, p, None) == shm.SHM_ERR_INVALID_ARG
    fl = lambda *a: call("shm_fit_forward_loss_grad", *a)
    assert fl(p, 8, p, p, p, 0, 1.0, p, None) == shm.SHM_OK
    assert fl(p, 0, p, p, p, 10, 1.0, p, None) == shm.SHM_ERR_INVALID_ARG
    assert fl(p, 8, p, p, p, -1, 1.0, p, None) == shm.SHM_ERR_INVALID_ARG
    assert fl(None, 8, p, p, p, 10, 1.0, p, None) == shm.SHM_ERR_INVALID_ARG
    assert fl(mis, 8, p, p, p, 10, 1.0, p, None) == shm.SHM_ERR_INVALID_ARG
    assert fl(p, 8, p, p, p, 10, float("inf"), p, None) == shm.SHM_ERR_INVALID_ARG
    ad = lambda *a: call("shm_adam_step", *a)
    ok = (0.9, 0.999, 1e-8)
    assert ad(p, p, p, p, 0, 1, 1e-3, 1e-3, *ok, None) == shm.SHM_OK
    assert ad(p, p, p, p, 10, 0, 1e-3, 1e-3, *ok, None) == shm.SHM_ERR_INVALID_ARG       # step >= 1
    assert ad(p, p, p, p, -1, 1, 1e-3, 1e-3, *ok, None) == shm.SHM_ERR_INVALID_ARG
    for b1, b2, eps in ((1.0, 0.999, 1e-8), (0.9, -0.1, 1e-8), (0.9, 0.999, 0.0), (0.9, 0.999, float("inf"))):
        assert ad(p, p, p, p, 10, 1, 1e-3, 1e-3, b1, b2, eps, None) == shm.SHM_ERR_INVALID_ARG
    assert ad(p, p, p, p, 10, 1, float("nan"), 1e-3, *ok, None) == shm.SHM_ERR_INVALID_ARG
    assert ad(p, None, p, p, 10, 1, 1e-3, 1e-3, *ok, None) == shm.SHM_ERR_INVALID_ARG
    assert ad(p, p, mis, p, 10, 1, 1e-3, 1e-3, *ok, None) == shm.SHM_ERR_INVALID_ARG


def test_fit_step_validation():
    """The fused fitting step refuses, before any launch: overlapping LUT and
    moment buffers (the update goes to a second LUT), a short or misaligned
    workspace, bad hyper-parameters and null or misaligned buffers."""
    N, Q = 8, 1000
    lut_bytes = 6 * (N + 2) ** 2 * 16
    a, b, m, v = (ctypes.c_void_p(k << 20) for k in (1, 2, 3, 4))
    ws_bytes = shm.lib().shm_backward_workspace(N, 1, Q)
    ws = ctypes.c_void_p(16 << 20)
    d = ctypes.c_void_p(32 << 20)
    ok = (1e-3, 1e-3, 0.9, 0.999, 1e-8)
    fs = lambda lin, lout, mm, vv, n=N, q=Q, wv=1.0, step=1, hp=ok, w=ws, wb=ws_bytes, dd=d, sr=1: call(
        "shm_fit_step", lin, lout, mm, vv, n, dd, dd, dd, q, wv, step, *hp, w, wb, sr, None)
    assert fs(a, b, m, v, sr=3) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, b, m, v, sr=-1) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, a, m, v) == shm.SHM_ERR_INVALID_ARG                                   # in place
    assert fs(a, ctypes.c_void_p((1 << 20) + lut_bytes - 16), m, v) == shm.SHM_ERR_INVALID_ARG  # overlap
    assert fs(a, b, m, m) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, b, a, v) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, b, m, v, wb=ws_bytes - 1) == shm.SHM_ERR_WORKSPACE
    assert fs(a, b, m, v, w=ctypes.c_void_p((16 << 20) + 16)) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, b, m, v, n=0) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, b, m, v, q=-1) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, b, m, v, wv=float("nan")) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, b, m, v, step=0) == shm.SHM_ERR_INVALID_ARG
    for hp in ((1e-3, 1e-3, 1.0, 0.999, 1e-8), (1e-3, 1e-3, 0.9, 0.999, 0.0), (float("inf"), 1e-3, 0.9, 0.999, 1e-8)):
        assert fs(a, b, m, v, hp=hp) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, None, m, v) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, b, m, v, dd=None) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, b, ctypes.c_void_p((3 << 20) + 4), v) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, b, m, v, wv=-1.0) == shm.SHM_ERR_INVALID_ARG
    assert fs(a, b, m, m) == shm.SHM_ERR_INVALID_ARG and "overlap" in shm.shm_last_error()


def test_size_products_do_not_overflow():
    """Object x query counts whose product would overflow 64 bits are
    refused on the host (no launch)."""
    p = ctypes.c_void_p(256)
    big = 1 << 40
    assert shm.lib().shm_backward_workspace(8, big, big) == 0
    assert call("shm_query_value_grad", p, 0, 0, 8, 1 << 62, p, 1 << 62, p, None, None) == shm.SHM_ERR_UNSUPPORTED
    assert call("shm_cell_keys", 8, big, p, big, p, None) == shm.SHM_ERR_UNSUPPORTED
    assert call("shm_backward_sort", 8, big, p, big, p, 1 << 30, None) == shm.SHM_ERR_UNSUPPORTED
    huge = 1 << 60
    assert call("shm_bake_fd", p, 8, huge, 0, p, None) == shm.SHM_ERR_UNSUPPORTED
    assert call("shm_lut_to_cells", p, 0, 8, huge, p, None) == shm.SHM_ERR_UNSUPPORTED
    assert call("shm_bake_sh_lut", p, 4, 8, huge, 0, p, p, 1 << 30, None) == shm.SHM_ERR_UNSUPPORTED


def test_gather_footprints_validation():
    p = ctypes.c_void_p(256)
    gf = lambda *a: call("shm_gather_footprints", *a)
    assert gf(p, 0, 0, 8, 1, p, 0, p, None) == shm.SHM_OK       # nothing to gather
    assert gf(p, 2, 0, 8, 1, p, 10, p, None) == shm.SHM_ERR_INVALID_ARG
    assert gf(p, 0, 2, 8, 1, p, 10, p, None) == shm.SHM_ERR_INVALID_ARG
    assert gf(p, 0, 0, 0, 1, p, 10, p, None) == shm.SHM_ERR_INVALID_ARG
    assert gf(p, 0, 0, 8, -1, p, 10, p, None) == shm.SHM_ERR_INVALID_ARG
    assert gf(p, 0, 0, 8, 1, p, 10, None, None) == shm.SHM_ERR_INVALID_ARG
    assert gf(p, 0, 0, 8, 1, p, 10, ctypes.c_void_p(264), None) == shm.SHM_ERR_INVALID_ARG  # foot not 16 B aligned
    assert gf(p, 0, 0, 8, 1 << 40, p, 1 << 40, p, None) == shm.SHM_ERR_UNSUPPORTED


def test_count_invalid_validation():
    p = ctypes.c_void_p(256)
    ci = lambda *a: call("shm_count_invalid", *a)
    assert ci(p, 0, p, None) == shm.SHM_OK             # nothing to count
    assert ci(p, -1, p, None) == shm.SHM_ERR_INVALID_ARG
    assert ci(p, 10, None, None) == shm.SHM_ERR_INVALID_ARG
    assert ci(p, 10, ctypes.c_void_p(260), None) == shm.SHM_ERR_INVALID_ARG   # count not 8-byte aligned
    assert ci(None, 10, p, None) == shm.SHM_ERR_INVALID_ARG
    assert ci(p, 1 << 62, p, None) == shm.SHM_ERR_UNSUPPORTED


def test_hip_error_is_reported_without_a_gpu():
    """With no GPU visible, calls whose arguments pass the host checks reach
    a launch (or a plan's device allocation), which the HIP runtime refuses:
    the entry point returns SHM_ERR_HIP and shm_last_error names the failing
    call.  Never run where a GPU is visible (the pointers are not real)."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible: this check must not launch on it")
    p = ctypes.c_void_p(1 << 20)
    assert call("shm_query_value_grad", p, 0, 0, 8, 1, p, 64, p, None, None) == shm.SHM_ERR_HIP
    assert "no ROCm-capable device" in shm.shm_last_error() or "launch" in shm.shm_last_error()
    assert call("shm_lut_rmax", p, 0, 8, 1, p, None) == shm.SHM_ERR_HIP
    assert shm.shm_last_error()
    # a valid call with nothing to do still succeeds: the error is not sticky
    assert call("shm_query_value_grad", p, 0, 0, 8, 1, p, 0, p, None, None) == shm.SHM_OK
    assert shm.shm_last_error() == ""


def test_probe_argument_validation():
    p = ctypes.c_void_p(256)
    assert call("shm_probe_gather", p, 4096, 4, 256, 48, 1, 0, None, p, None) == shm.SHM_ERR_INVALID_ARG  # req size
    assert "req_bytes" in shm.shm_last_error()
    assert call("shm_probe_gather", p, 4096, 4, 256, 64, 1, 4, None, p, None) == shm.SHM_ERR_INVALID_ARG   # flags
    assert call("shm_probe_gather", p, 4100, 4, 256, 64, 1, 0, None, p, None) == shm.SHM_ERR_INVALID_ARG  # region % 16
    assert call("shm_probe_gather", p, 32, 4, 256, 64, 1, 0, None, p, None) == shm.SHM_ERR_INVALID_ARG    # region < req
    assert call("shm_probe_gather", ctypes.c_void_p(8), 4096, 4, 256, 64, 1, 0, None, p, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_probe_gather", p, 4096, 4, 256, 64, 1, 0, None, None, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_probe_gather", p, 4096, 4, 256, 64, 1, shm.SHM_PROBE_DIRS, None, p, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_probe_gather", p, 4096, 1 << 40, 1 << 40, 64, 1, 0, None, p, None) == shm.SHM_ERR_UNSUPPORTED
    assert call("shm_probe_gather", p, 4096, 0, 256, 64, 1, 0, None, None, None) == shm.SHM_OK  # empty
    assert call("shm_probe_stream_read", p, 100, p, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_probe_stream_read", p, 0, None, None) == shm.SHM_OK
    fl = ctypes.c_double(-1.0)
    mf = lambda w, c, it, f=ctypes.byref(fl), sk=p: call("shm_probe_mfma_f32", w, c, it, f, sk, None)
    for args in ((0, 4, 10), (9, 4, 10), (2, 3, 10), (2, 16, 10), (2, 4, 0)):
        assert mf(*args) == shm.SHM_ERR_INVALID_ARG, args
    assert mf(2, 4, 10, f=None) == shm.SHM_ERR_INVALID_ARG
    assert mf(2, 4, 10, sk=None) == shm.SHM_ERR_INVALID_ARG
    assert mf(2, 4, 10, sk=ctypes.c_void_p(260)) == shm.SHM_ERR_INVALID_ARG
    assert fl.value == -1.0  # nothing written on refusal
    assert call("shm_plan_probe", None, p, p, p, 1, None) == shm.SHM_ERR_INVALID_ARG  # no plan, no device call
    assert "null plan" in shm.shm_last_error()


def test_query_objects_argument_validation():
    """The plan-free object query validates on the host before any launch."""
    p = ctypes.c_void_p(256)
    ws_need = shm.shm_query_objects_workspace(10)
    assert ws_need == 88  # n_obj + 1 int64 tile offsets
    f = "shm_query_objects"
    assert call(f, p, 5, 0, p, 10, p, p, None, p, ws_need, None) == shm.SHM_ERR_INVALID_ARG  # dtype
    assert call(f, p, 0, 7, p, 10, p, p, None, p, ws_need, None) == shm.SHM_ERR_INVALID_ARG  # layout
    assert call(f, p, 0, 0, p, -1, p, p, None, p, ws_need, None) == shm.SHM_ERR_INVALID_ARG
    assert call(f, p, 0, 0, None, 10, p, p, None, p, ws_need, None) == shm.SHM_ERR_INVALID_ARG
    assert call(f, p, 0, 0, p, 10, p, p, None, None, ws_need, None) == shm.SHM_ERR_INVALID_ARG
    assert call(f, p, 0, 0, p, 10, p, p, None, p, ws_need - 1, None) == shm.SHM_ERR_WORKSPACE
    assert "workspace" in shm.shm_last_error()
    assert call(f, p, 0, 0, ctypes.c_void_p(260), 10, p, p, None, p, ws_need, None) == shm.SHM_ERR_INVALID_ARG
    assert call(f, ctypes.c_void_p(264), 0, 1, p, 10, p, p, None, p, ws_need, None) == shm.SHM_ERR_INVALID_ARG
    assert call(f, None, 0, 0, None, 0, None, None, None, None, 0, None) == shm.SHM_OK  # no objects


def test_plan_backward_argument_validation():
    p = ctypes.c_void_p(256)
    assert call("shm_plan_backward_sort", None, p, None) == shm.SHM_ERR_INVALID_ARG
    assert "null plan" in shm.shm_last_error()
    assert call("shm_plan_backward", None, p, p, p, p, p, None) == shm.SHM_ERR_INVALID_ARG


def test_bake_noalloc_argument_validation():
    """The no-allocation bake validates like the workspace bake and refuses a
    basis table larger than its scratch before touching a device."""
    p = ctypes.c_void_p(256)
    assert call("shm_bake_sh_lut_noalloc", p, 16, 64, 1, 0, p, None) == shm.SHM_ERR_UNSUPPORTED
    assert "scratch" in shm.shm_last_error()
    assert shm.shm_bake_sh_lut_workspace(16, 64) > shm.SHM_BAKE_NOALLOC_MAX_BYTES >= shm.shm_bake_sh_lut_workspace(16, 32)
    assert call("shm_bake_sh_lut_noalloc", p, 17, 8, 1, 0, p, None) == shm.SHM_ERR_UNSUPPORTED
    assert call("shm_bake_sh_lut_noalloc", p, 4, 0, 1, 0, p, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_bake_sh_lut_noalloc", None, 4, 8, 1, 0, p, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_bake_sh_lut_noalloc", p, 4, 8, 1, 7, p, None) == shm.SHM_ERR_INVALID_ARG
    assert call("shm_bake_sh_lut_noalloc", None, 4, 8, 0, 0, None, None) == shm.SHM_OK
