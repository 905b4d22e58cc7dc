"""MI355X (gfx950) Spherical Hermite Maps: Python binding of libshm.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libshm.so`` (built from ``csrc/`` by ``build.py``).  PyTorch provides
device memory and streams.  There is no CPU fallback: if the library is not
built or no GPU is present the calls raise.

The functions named ``shm_*`` mirror the C ABI in ``include/shm.h`` one to
one (same names and arguments, tensors in place of device pointers); the
helpers below them allocate outputs and workspaces with torch.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshm.so")
# a host-only, sanitizer-instrumented build of the same sources
# (build.build_host_sanitized) can be loaded in its place for the host-side
# argument checks; it holds no device code
if os.environ.get("SHM_LIBRARY"):
    LIB_PATH = os.environ["SHM_LIBRARY"]

SHM_OK, SHM_ERR_INVALID_ARG, SHM_ERR_UNSUPPORTED, SHM_ERR_WORKSPACE, SHM_ERR_HIP = range(5)
SHM_F32, SHM_F16 = 0, 1
SHM_LAYOUT_TEXEL, SHM_LAYOUT_CELL = 0, 1
SHM_MAX_N, SHM_MAX_L, SHM_MAX_BOUND_BLOCKS = 1024, 16, 64
SHM_RECON_NEAREST, SHM_RECON_BILINEAR_FD, SHM_RECON_BICUBIC, SHM_RECON_FAST_BICUBIC_FD = 0, 1, 2, 3
SHM_SIGNED = 1
SHM_CELL_LUT = 2
SHM_PROBE_DIRS, SHM_PROBE_OUT = 1, 2
SHM_BAKE_NOALLOC_MAX_BYTES = 32 << 20  # scratch of shm_bake_sh_lut_noalloc
SHM_SORT_READY, SHM_SORT_READY_SPARSE = 1, 2


class ShmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libshm error {code}: {msg}")
        self.code = code


class shm_object(ctypes.Structure):
    _fields_ = [("lut_offset", ctypes.c_int64), ("N", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("q_begin", ctypes.c_int64), ("q_count", ctypes.c_int64)]


class shm_launch_shape(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("qpt", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("grid_per_cu", ctypes.c_int32)]

    def as_dict(self):
        return {"block": self.block, "qpt": self.qpt, "tile": self.tile, "grid_per_cu": self.grid_per_cu}


class shm_trace_params(ctypes.Structure):
    _fields_ = [("scale", ctypes.c_float), ("flags", ctypes.c_int32), ("n_march", ctypes.c_int32),
                ("n_bisect", ctypes.c_int32), ("n_newton", ctypes.c_int32), ("px_per_unit", ctypes.c_float),
                ("eps_px", ctypes.c_float), ("image_width", ctypes.c_int32), ("bound_blocks", ctypes.c_int32),
                ("bound_map", ctypes.c_void_p)]


_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t

# name -> (restype, argtypes)
SIGNATURES = {
    "shm_version": (ctypes.c_int, []),
    "shm_last_error": (ctypes.c_char_p, []),
    "shm_lut_elems": (_I64, [_I32, _I32]),
    "shm_bake_sh_lut_workspace": (_SZ, [_I32, _I32]),
    "shm_bake_sh_lut": (ctypes.c_int, [_VP, _I32, _I32, _I64, _I32, _VP, _VP, _SZ, _VP]),
    "shm_margin_dirs": (ctypes.c_int, [_I32, _VP, _VP]),
    "shm_bake_fd": (ctypes.c_int, [_VP, _I32, _I64, _I32, _VP, _VP]),
    "shm_lut_to_cells": (ctypes.c_int, [_VP, _I32, _I32, _I64, _VP, _VP]),
    "shm_query_value_grad": (ctypes.c_int, [_VP, _I32, _I32, _I32, _I64, _VP, _I64, _VP, _VP, _VP]),
    "shm_plan_create": (ctypes.c_int, [_VP, _I64, _I32, _I32, _VP, ctypes.POINTER(_VP)]),
    "shm_plan_autotune": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_char_p, _VP, ctypes.POINTER(shm_launch_shape)]),
    "shm_plan_set_shape": (ctypes.c_int, [_VP, ctypes.POINTER(shm_launch_shape)]),
    "shm_plan_launch": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "shm_plan_capture_graph": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "shm_plan_graph_launch": (ctypes.c_int, [_VP, _VP]),
    "shm_plan_work_items": (_I64, [_VP]),
    "shm_plan_destroy": (ctypes.c_int, [_VP]),
    "shm_backward_workspace": (_SZ, [_I32, _I64, _I64]),
    "shm_cell_keys": (ctypes.c_int, [_I32, _I64, _VP, _I64, _VP, _VP]),
    "shm_backward_sort": (ctypes.c_int, [_I32, _I64, _VP, _I64, _VP, _SZ, _VP]),
    "shm_query_backward": (ctypes.c_int, [_VP, _I32, _I64, _VP, _I64, _VP, _VP, _VP, _VP, _SZ, _I32, _VP]),
    "shm_backward_dense_tiles": (_I64, [_I32, _I64, _I64, _VP, _SZ, _VP]),
    "shm_trace_radial": (ctypes.c_int, [_VP, _I32, _I32, ctypes.POINTER(ctypes.c_float), ctypes.c_float, _VP, _VP,
                                        _I64, _I32, _I32, _I32, _VP, _VP, _VP, _VP]),
    "shm_trace_radial_ex": (ctypes.c_int, [_VP, _I32, _I32, ctypes.POINTER(ctypes.c_float), ctypes.c_float,
                                           ctypes.POINTER(shm_trace_params), _VP, _VP, _I64, _VP, _VP, _VP, _VP, _VP,
                                           _VP]),
    "shm_lut_rmax": (ctypes.c_int, [_VP, _I32, _I32, _I32, _VP, _VP]),
    "shm_query_scaled": (ctypes.c_int, [_VP, _I32, _I32, _I32, _I64, _VP, _I64, ctypes.c_float, _I32, _VP, _VP, _VP,
                                        _VP]),
    "shm_mip_level_workspace": (_SZ, [_I32]),
    "shm_mip_level": (ctypes.c_int, [_VP, _I32, _I32, _VP, _SZ, _VP, _VP]),
    "shm_mesh_radial_depth": (ctypes.c_int, [_VP, _I64, _VP, _I64, ctypes.POINTER(ctypes.c_float), _VP, _I64, _VP,
                                             _VP]),
    "shm_query_baseline": (ctypes.c_int, [_VP, _I32, _I64, _VP, _I64, _I32, _VP, _VP]),
    "shm_sh_eval": (ctypes.c_int, [_VP, _I32, _I64, _VP, _I64, _VP, _VP]),
    "shm_lut_bound_map": (ctypes.c_int, [_VP, _I32, _I32, _I32, _I32, _VP, _VP]),
    "shm_fit_loss_grad": (ctypes.c_int, [_VP, _VP, _VP, _VP, _I64, ctypes.c_float, _VP, _VP]),
    "shm_fit_forward_loss_grad": (ctypes.c_int, [_VP, _I32, _VP, _VP, _VP, _I64, ctypes.c_float, _VP, _VP]),
    "shm_adam_step": (ctypes.c_int, [_VP, _VP, _VP, _VP, _I64, _I64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, _VP]),
    "shm_count_invalid": (ctypes.c_int, [_VP, _I64, _VP, _VP]),
    "shm_cells_to_f16": (ctypes.c_int, [_VP, _I64, _VP, _VP]),
    "shm_gather_footprints": (ctypes.c_int, [_VP, _I32, _I32, _I32, _I64, _VP, _I64, _VP, _VP]),
    "shm_fit_step": (ctypes.c_int, [_VP, _VP, _VP, _VP, _I32, _VP, _VP, _VP, _I64, ctypes.c_float, _I64,
                                    ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    _VP, ctypes.c_size_t, _I32, _VP]),
    "shm_bake_sh_lut_noalloc": (ctypes.c_int, [_VP, _I32, _I32, _I64, _I32, _VP, _VP]),
    # memory-system probes (include/shm_probe.h)
    "shm_probe_gather": (ctypes.c_int, [_VP, _I64, _I64, _I64, _I32, ctypes.c_uint32, _I32, _VP, _VP, _VP]),
    "shm_probe_stream_read": (ctypes.c_int, [_VP, _I64, _VP, _VP]),
    "shm_probe_mfma_f32": (ctypes.c_int, [_I32, _I32, _I64, ctypes.POINTER(ctypes.c_double), _VP, _VP]),
    "shm_query_objects_workspace": (_SZ, [_I64]),
    "shm_plan_backward_sort": (ctypes.c_int, [_VP, _VP, _VP]),
    "shm_plan_backward": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "shm_query_objects": (ctypes.c_int, [_VP, _I32, _I32, _VP, _I64, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "shm_plan_probe": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_uint32, _VP]),
}

_lib = None


def lib():
    """Load libshm.so (fails loudly if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2602_20063_amd/build.py (or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != SHM_OK:
        raise ShmError(rc, lib().shm_last_error().decode())
    return rc


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libshm takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libshm takes contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(t):
    if t.dtype == torch.float32:
        return SHM_F32
    if t.dtype == torch.float16:
        return SHM_F16
    raise ValueError(f"LUT dtype must be float32 or float16, got {t.dtype}")


def _need(t, dtype, name):
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")


def _fits(t, nbytes, name):
    """The C ABI takes bare pointers: refuse a tensor smaller than the bytes
    the call will read or write there, before anything is launched."""
    if t is not None and nbytes > 0 and t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name} holds {t.numel() * t.element_size()} bytes; the call accesses {nbytes}")


def _dbytes(dtype_code):
    return 2 if dtype_code == SHM_F16 else 4


def _lut_bytes(N, layout, dtype_code, n_obj=1):
    per = 6 * (N + 2) ** 2 * 4 if layout == SHM_LAYOUT_TEXEL else 6 * (N + 1) ** 2 * 16
    return max(n_obj, 0) * per * _dbytes(dtype_code)


# ---------------------------------------------------------------------------
# one-to-one mirrors of the C ABI
# ---------------------------------------------------------------------------
def shm_version():
    return lib().shm_version()


def shm_last_error():
    return lib().shm_last_error().decode()


def shm_lut_elems(N, layout=SHM_LAYOUT_TEXEL):
    return lib().shm_lut_elems(N, layout)


def shm_bake_sh_lut_workspace(L, N):
    return lib().shm_bake_sh_lut_workspace(L, N)


def shm_bake_sh_lut(coeffs, L, N, n_obj, out_dtype, lut_out, ws, stream=None):
    _need(coeffs, torch.float32, "coeffs")
    _fits(coeffs, max(n_obj, 0) * (L + 1) ** 2 * 4, "coeffs")
    _fits(lut_out, _lut_bytes(N, SHM_LAYOUT_TEXEL, out_dtype, n_obj), "lut_out")
    return _check(lib().shm_bake_sh_lut(_ptr(coeffs), L, N, n_obj, out_dtype, _ptr(lut_out), _ptr(ws),
                                        ws.numel() * ws.element_size(), _stream(stream)))


def shm_bake_sh_lut_noalloc(coeffs, L, N, n_obj, out_dtype, lut_out, stream=None):
    """The SH bake without a workspace (the library's scratch array)."""
    _need(coeffs, torch.float32, "coeffs")
    _fits(coeffs, max(n_obj, 0) * (L + 1) ** 2 * 4, "coeffs")
    _fits(lut_out, _lut_bytes(N, SHM_LAYOUT_TEXEL, out_dtype, n_obj), "lut_out")
    return _check(lib().shm_bake_sh_lut_noalloc(_ptr(coeffs), L, N, n_obj, out_dtype, _ptr(lut_out), _stream(stream)))


def shm_margin_dirs(N, dirs, stream=None):
    _need(dirs, torch.float32, "dirs")
    _fits(dirs, 6 * (N + 4) ** 2 * 12, "dirs")
    return _check(lib().shm_margin_dirs(N, _ptr(dirs), _stream(stream)))


def shm_bake_fd(samples, N, n_obj, out_dtype, lut_out, stream=None):
    _need(samples, torch.float32, "samples")
    _fits(samples, max(n_obj, 0) * 6 * (N + 4) ** 2 * 4, "samples")
    _fits(lut_out, _lut_bytes(N, SHM_LAYOUT_TEXEL, out_dtype, n_obj), "lut_out")
    return _check(lib().shm_bake_fd(_ptr(samples), N, n_obj, out_dtype, _ptr(lut_out), _stream(stream)))


def shm_lut_to_cells(lut_texel, dtype, N, n_obj, lut_cell, stream=None):
    _fits(lut_texel, _lut_bytes(N, SHM_LAYOUT_TEXEL, dtype, n_obj), "lut_texel")
    _fits(lut_cell, _lut_bytes(N, SHM_LAYOUT_CELL, dtype, n_obj), "lut_cell")
    return _check(lib().shm_lut_to_cells(_ptr(lut_texel), dtype, N, n_obj, _ptr(lut_cell), _stream(stream)))


def shm_query_value_grad(lut, dtype, layout, N, n_obj, dirs, q_per_obj, out, normal=None, stream=None):
    _need(dirs, torch.float32, "dirs")
    _need(out, torch.float32, "out")
    Q = max(n_obj, 0) * max(q_per_obj, 0)
    if Q:
        _fits(lut, _lut_bytes(N, layout, dtype, n_obj), "lut")
    _fits(dirs, Q * 12, "dirs")
    _fits(out, Q * 16, "out")
    _fits(normal, Q * 12, "normal")
    return _check(lib().shm_query_value_grad(_ptr(lut), dtype, layout, N, n_obj, _ptr(dirs), q_per_obj, _ptr(out),
                                             _ptr(normal), _stream(stream)))


def shm_query_objects_workspace(n_obj):
    return lib().shm_query_objects_workspace(n_obj)


def shm_query_objects(lut, dtype, layout, objs, n_obj, dirs, out, normal, ws, stream=None):
    """objs: device tensor holding n_obj shm_object records (objects_tensor)."""
    _need(dirs, torch.float32, "dirs")
    _need(out, torch.float32, "out")
    _fits(objs, max(n_obj, 0) * ctypes.sizeof(shm_object), "objs")
    _fits(ws, shm_query_objects_workspace(n_obj) if n_obj > 0 else 0, "ws")
    return _check(lib().shm_query_objects(_ptr(lut), dtype, layout, _ptr(objs), n_obj, _ptr(dirs), _ptr(out),
                                          _ptr(normal), _ptr(ws), ws.numel() * ws.element_size() if ws is not None
                                          else 0, _stream(stream)))


def objects_tensor(objs, device="cuda"):
    """shm_object records [(lut_offset, N, q_begin, q_count), ...] as a
    device tensor (int64 [n, 4]; N in the low half of the second word)."""
    rows = [[int(off), int(N) & 0xFFFFFFFF, int(qb), int(qc)] for (off, N, qb, qc) in objs]
    return torch.tensor(rows, dtype=torch.int64).reshape(-1, 4).to(device)


def query_objects(lut, dirs, objs, dtype=None, layout=SHM_LAYOUT_TEXEL, normals=False, out=None, stream=None):
    """Value + gradient of uneven objects without a plan: objs as for Plan
    ((lut_offset, N, q_begin, q_count) per object, ranges disjoint); rows of
    out outside every range are left as they were."""
    dtype = _dtype_code(lut) if dtype is None else dtype
    rows = max((int(qb) + int(qc) for (_, _, qb, qc) in objs if int(qc) > 0), default=0)
    need = max((int(off) * _dbytes(dtype) + _lut_bytes(int(N), layout, dtype) for (off, N, _, qc) in objs
                if int(qc) > 0), default=0)
    _fits(lut, need, "lut")
    _fits(dirs, rows * 12, "dirs")
    if out is None:
        out = torch.empty((dirs.shape[0], 4), dtype=torch.float32, device=dirs.device)
    _fits(out, rows * 16, "out")
    nrm = torch.empty((dirs.shape[0], 3), dtype=torch.float32, device=dirs.device) if normals else None
    od = objects_tensor(objs, dirs.device)
    ws = torch.empty(max(shm_query_objects_workspace(len(objs)), 8), dtype=torch.uint8, device=dirs.device)
    shm_query_objects(lut, dtype, layout, od, len(objs), dirs, out, nrm, ws, stream)
    return (out, nrm) if normals else out


def shm_probe_gather(base, region_bytes, n_regions, per_region, req_bytes, seed, flags, dirs, out, stream=None):
    """Random gathers of req_bytes inside regions of base (see shm_probe.h),
    with the query's streamed directions (SHM_PROBE_DIRS) and/or 16 B results
    (SHM_PROBE_OUT)."""
    n = max(n_regions, 0) * max(per_region, 0)
    if n and req_bytes:
        _fits(base, n_regions * region_bytes, "base")
    _fits(dirs, n * 12 if flags & SHM_PROBE_DIRS else 0, "dirs")
    _fits(out, n * 16 if flags & SHM_PROBE_OUT else (16 if n else 0), "out")
    return _check(lib().shm_probe_gather(_ptr(base), region_bytes, n_regions, per_region, req_bytes, seed & 0xFFFFFFFF,
                                         flags, _ptr(dirs), _ptr(out), _stream(stream)))


def shm_probe_stream_read(base, nbytes, sink, stream=None):
    _fits(base, nbytes, "base")
    _fits(sink, 16 if nbytes > 0 else 0, "sink")
    return _check(lib().shm_probe_stream_read(_ptr(base), nbytes, _ptr(sink), _stream(stream)))


def shm_probe_mfma_f32(waves_per_simd, chains, iters, sink, stream=None):
    """Launch the FP32 matrix-core probe; returns the launch's flop count."""
    _fits(sink, 16, "sink")
    fl = ctypes.c_double(0.0)
    _check(lib().shm_probe_mfma_f32(waves_per_simd, chains, iters, ctypes.byref(fl), _ptr(sink), _stream(stream)))
    return fl.value


def shm_backward_workspace(N, n_obj, q_per_obj):
    return lib().shm_backward_workspace(N, n_obj, q_per_obj)


def shm_cell_keys(N, n_obj, dirs, q_per_obj, keys, stream=None):
    _need(keys, torch.int32, "keys (uint32 bits stored as int32)")
    _fits(dirs, max(n_obj, 0) * max(q_per_obj, 0) * 12, "dirs")
    _fits(keys, max(n_obj, 0) * max(q_per_obj, 0) * 4, "keys")
    return _check(lib().shm_cell_keys(N, n_obj, _ptr(dirs), q_per_obj, _ptr(keys), _stream(stream)))


def shm_backward_sort(N, n_obj, dirs, q_per_obj, ws, stream=None):
    _fits(dirs, max(n_obj, 0) * max(q_per_obj, 0) * 12, "dirs")
    return _check(lib().shm_backward_sort(N, n_obj, _ptr(dirs), q_per_obj, _ptr(ws), ws.numel() * ws.element_size(),
                                          _stream(stream)))


def _sort_ready(x):
    """sort_ready as the library takes it: False/True -> 0/SHM_SORT_READY,
    integers unchanged (0, SHM_SORT_READY or SHM_SORT_READY_SPARSE)."""
    return int(bool(x)) if isinstance(x, bool) else int(x)


def shm_backward_dense_tiles(N, n_obj, q_per_obj, ws, stream=None):
    n = lib().shm_backward_dense_tiles(N, n_obj, q_per_obj, _ptr(ws), ws.numel() * ws.element_size(), _stream(stream))
    if n < 0:
        raise ShmError(SHM_ERR_INVALID_ARG, lib().shm_last_error().decode())
    return int(n)


def shm_query_backward(lut, N, n_obj, dirs, q_per_obj, grad_out, grad_lut, grad_dirs, ws, sort_ready, stream=None):
    Q = max(n_obj, 0) * max(q_per_obj, 0)
    lb = _lut_bytes(N, SHM_LAYOUT_TEXEL, SHM_F32, n_obj)
    _fits(lut, lb, "lut")
    _fits(dirs, Q * 12, "dirs")
    _fits(grad_out, Q * 16, "grad_out")
    _fits(grad_lut, lb, "grad_lut")
    _fits(grad_dirs, Q * 12, "grad_dirs")
    return _check(lib().shm_query_backward(_ptr(lut), N, n_obj, _ptr(dirs), q_per_obj, _ptr(grad_out), _ptr(grad_lut),
                                           _ptr(grad_dirs), _ptr(ws), ws.numel() * ws.element_size(),
                                           _sort_ready(sort_ready), _stream(stream)))


def _fits_rays(P, ray_o, ray_d, t_out, out, normal, sign=None, evals=None):
    P = max(P, 0)
    for t, b, name in ((ray_o, 12, "ray_o"), (ray_d, 12, "ray_d"), (t_out, 4, "t_out"), (out, 16, "out"),
                       (normal, 12, "normal"), (sign, 1, "sign"), (evals, 1, "evals")):
        _fits(t, P * b, name)


def shm_trace_radial(lut, dtype, N, center, rmax, ray_o, ray_d, P, n_march, n_bisect, n_newton, t_out, out,
                     normal=None, stream=None):
    _fits(lut, _lut_bytes(N, SHM_LAYOUT_TEXEL, dtype) if P > 0 else 0, "lut")
    _fits_rays(P, ray_o, ray_d, t_out, out, normal)
    c = (ctypes.c_float * 3)(*[float(x) for x in center])
    return _check(lib().shm_trace_radial(_ptr(lut), dtype, N, c, float(rmax), _ptr(ray_o), _ptr(ray_d), P, n_march,
                                         n_bisect, n_newton, _ptr(t_out), _ptr(out), _ptr(normal), _stream(stream)))


def shm_trace_radial_ex(lut, dtype, N, center, rmax, params, ray_o, ray_d, P, t_out, out, normal=None, sign=None,
                        evals=None, stream=None):
    layout = SHM_LAYOUT_CELL if params.flags & SHM_CELL_LUT else SHM_LAYOUT_TEXEL
    _fits(lut, _lut_bytes(N, layout, dtype) if P > 0 else 0, "lut")
    _fits_rays(P, ray_o, ray_d, t_out, out, normal, sign, evals)
    c = (ctypes.c_float * 3)(*[float(x) for x in center])
    return _check(lib().shm_trace_radial_ex(_ptr(lut), dtype, N, c, float(rmax), ctypes.byref(params), _ptr(ray_o),
                                            _ptr(ray_d), P, _ptr(t_out), _ptr(out), _ptr(normal), _ptr(sign),
                                            _ptr(evals), _stream(stream)))


def shm_lut_rmax(lut, dtype, N, flags, rmax_out, stream=None):
    return _check(lib().shm_lut_rmax(_ptr(lut), dtype, N, flags, _ptr(rmax_out), _stream(stream)))


def shm_query_scaled(lut, dtype, layout, N, n_obj, dirs, q_per_obj, scale, flags, out, normal=None, sign=None,
                     stream=None):
    Q = max(n_obj, 0) * max(q_per_obj, 0)
    if Q:
        _fits(lut, _lut_bytes(N, layout, dtype, n_obj), "lut")
    _fits(dirs, Q * 12, "dirs")
    _fits(out, Q * 16, "out")
    _fits(normal, Q * 12, "normal")
    _fits(sign, Q, "sign")
    return _check(lib().shm_query_scaled(_ptr(lut), dtype, layout, N, n_obj, _ptr(dirs), q_per_obj, float(scale),
                                         flags, _ptr(out), _ptr(normal), _ptr(sign), _stream(stream)))


def shm_mesh_radial_depth(verts, n_verts, tris, n_tris, center, dirs, P, depth, stream=None):
    c = (ctypes.c_float * 3)(*[float(x) for x in center])
    return _check(lib().shm_mesh_radial_depth(_ptr(verts), n_verts, _ptr(tris), n_tris, c, _ptr(dirs), P,
                                              _ptr(depth), _stream(stream)))


def _fits_fit(Q, dirs, target_r, target_n):
    Q = max(Q, 0)
    _fits(dirs, Q * 12, "dirs")
    _fits(target_r, Q * 4, "target_r")
    _fits(target_n, Q * 12, "target_n")


def shm_fit_loss_grad(out, dirs, target_r, target_n, Q, w_value, grad, stream=None):
    _fits_fit(Q, dirs, target_r, target_n)
    _fits(out, max(Q, 0) * 16, "out")
    _fits(grad, max(Q, 0) * 16, "grad")
    return _check(lib().shm_fit_loss_grad(_ptr(out), _ptr(dirs), _ptr(target_r), _ptr(target_n), Q, float(w_value),
                                          _ptr(grad), _stream(stream)))


def shm_fit_forward_loss_grad(lut, N, dirs, target_r, target_n, Q, w_value, grad, stream=None):
    _fits(lut, _lut_bytes(N, SHM_LAYOUT_TEXEL, SHM_F32) if Q > 0 else 0, "lut")
    _fits_fit(Q, dirs, target_r, target_n)
    _fits(grad, max(Q, 0) * 16, "grad")
    return _check(lib().shm_fit_forward_loss_grad(_ptr(lut), N, _ptr(dirs), _ptr(target_r), _ptr(target_n), Q,
                                                  float(w_value), _ptr(grad), _stream(stream)))


def shm_adam_step(param, grad, m, v, n4, step, lr_value, lr_deriv, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    for t, name in ((param, "param"), (grad, "grad"), (m, "m"), (v, "v")):
        _fits(t, max(n4, 0) * 16, name)
    return _check(lib().shm_adam_step(_ptr(param), _ptr(grad), _ptr(m), _ptr(v), n4, step, float(lr_value),
                                      float(lr_deriv), float(beta1), float(beta2), float(eps), _stream(stream)))


def shm_gather_footprints(lut, dtype, layout, N, n_obj, dirs, q_per_obj, foot, stream=None):
    _need(dirs, torch.float32, "dirs")
    _need(foot, torch.float32, "foot")
    Q = max(n_obj, 0) * max(q_per_obj, 0)
    if Q:
        _fits(lut, _lut_bytes(N, layout, dtype, n_obj), "lut")
    _fits(dirs, Q * 12, "dirs")
    _fits(foot, Q * 64, "foot")
    return _check(lib().shm_gather_footprints(_ptr(lut), dtype, layout, N, n_obj, _ptr(dirs), q_per_obj, _ptr(foot),
                                              _stream(stream)))


def shm_count_invalid(dirs, Q, count, stream=None):
    _need(count, torch.int64, "count")
    _fits(dirs, max(Q, 0) * 12, "dirs")
    _fits(count, 8, "count")
    return _check(lib().shm_count_invalid(_ptr(dirs), Q, _ptr(count), _stream(stream)))


def count_invalid(dirs, stream=None):
    """Number of directions every query answers with NaN (zero vector, NaN or
    Inf component); synchronises."""
    c = torch.zeros(1, dtype=torch.int64, device=dirs.device)
    shm_count_invalid(dirs.contiguous(), dirs.shape[0], c, stream)
    return int(c.item())


def shm_fit_step(lut_in, lut_out, m, v, N, dirs, target_r, target_n, Q, w_value, step, lr_value, lr_deriv,
                 beta1, beta2, eps, ws, sort_ready, stream=None):
    for t, name in ((lut_in, "lut_in"), (lut_out, "lut_out"), (m, "m"), (v, "v")):
        _need(t, torch.float32, name)
        _fits(t, _lut_bytes(N, SHM_LAYOUT_TEXEL, SHM_F32), name)
    _fits_fit(Q, dirs, target_r, target_n)
    return _check(lib().shm_fit_step(_ptr(lut_in), _ptr(lut_out), _ptr(m), _ptr(v), N, _ptr(dirs), _ptr(target_r),
                                     _ptr(target_n), Q, float(w_value), step, float(lr_value), float(lr_deriv),
                                     float(beta1), float(beta2), float(eps), _ptr(ws), ws.numel() * ws.element_size(),
                                     _sort_ready(sort_ready), _stream(stream)))


class LutFit:
    """Fits one FP32 TEXEL LUT (face size N) to target radii and normals at
    fixed directions with Adam (value + normal objective, value term
    weighted by w_value; directions sorted by cell once), every step in this
    library's kernels.

    fused=True: one shm_fit_step kernel per step, alternating two LUT
    buffers; `lut` is the current one.  fused=False: the three-kernel step
    (forward query fused with the loss gradient, LUT-only backward, Adam
    update), updating the given LUT in place."""

    def __init__(self, lut, dirs, target_r, target_n, w_value=1.0, lr_value=1e-3, lr_deriv=1e-3, betas=(0.9, 0.999),
                 eps=1e-8, fused=True, stream=None):
        self.N = lut_n(lut)
        self.dirs = dirs
        self.tr, self.tn = target_r.contiguous(), target_n.contiguous()
        self.Q = dirs.shape[0]
        self.w_value, self.lr_value, self.lr_deriv = w_value, lr_value, lr_deriv
        self.betas, self.eps = betas, eps
        self.fused = fused
        self.bctx = BackwardContext(self.N, 1, dirs, self.Q, stream, check_dense=True)
        dev = lut.device
        self.bufs = [lut, torch.empty_like(lut)] if fused else [lut]
        self.cur = 0
        if not fused:
            self.g = torch.empty((self.Q, 4), device=dev)
            self.grad = torch.empty_like(lut)
        self.m = torch.zeros_like(lut)
        self.v = torch.zeros_like(lut)
        self.t = 0

    @property
    def lut(self):
        return self.bufs[self.cur]

    def state_dict(self):
        """Checkpoint of the fit: current LUT, Adam moments and step count
        (tensors cloned; save with torch.save)."""
        return {"lut": self.lut.clone(), "m": self.m.clone(), "v": self.v.clone(), "t": int(self.t)}

    def load_state_dict(self, state):
        """Resume from state_dict(): the following steps continue the fit
        exactly (the same bits as never having stopped)."""
        if state["lut"].shape != self.lut.shape or state["m"].shape != self.m.shape:
            raise ValueError("checkpoint of a LUT of another shape")
        self.lut.copy_(state["lut"])
        self.m.copy_(state["m"])
        self.v.copy_(state["v"])
        self.t = int(state["t"])

    def step(self, stream=None):
        self.t += 1
        N, Q = self.N, self.Q
        b1, b2 = self.betas
        if self.fused:
            nxt = 1 - self.cur
            shm_fit_step(self.bufs[self.cur], self.bufs[nxt], self.m, self.v, N, self.dirs, self.tr, self.tn, Q,
                         self.w_value, self.t, self.lr_value, self.lr_deriv, b1, b2, self.eps, self.bctx.ws,
                         self.bctx.sort_ready, stream)
            self.cur = nxt
            return
        lut = self.lut
        shm_fit_forward_loss_grad(lut, N, self.dirs, self.tr, self.tn, Q, self.w_value, self.g, stream)
        shm_query_backward(lut, N, 1, self.dirs, Q, self.g, self.grad, None, self.bctx.ws, self.bctx.sort_ready,
                           stream)
        shm_adam_step(lut, self.grad, self.m, self.v, lut.numel() // 4, self.t, self.lr_value, self.lr_deriv, b1, b2,
                      self.eps, stream)


def mesh_radial_depth(verts, tris, center, dirs, stream=None):
    """verts [V, 3] FP32, tris [T, 3] int32 (device), center (3 floats),
    dirs [P, 3] -> depth [P] FP32."""
    verts = verts.contiguous()
    tris = tris.contiguous()
    P = dirs.shape[0]
    depth = torch.empty(P, dtype=torch.float32, device=dirs.device)
    shm_mesh_radial_depth(verts, verts.shape[0], tris, tris.shape[0], center, dirs, P, depth, stream)
    return depth


def bake_mesh(verts, tris, center, N, dtype=torch.float32, stream=None):
    """Impostor LUT of a mesh: radial depth on the margin grid of face size
    N, then the finite-difference bake.  LUT [1, 6, N+2, N+2, 4]."""
    d = margin_dirs(N, device=verts.device, stream=stream).reshape(-1, 3)
    depth = mesh_radial_depth(verts, tris, center, d, stream)
    return bake_fd(depth.reshape(1, 6, N + 4, N + 4), N, dtype=dtype, stream=stream)


def shm_mip_level_workspace(N):
    return lib().shm_mip_level_workspace(N)


def shm_mip_level(lut, N, mode, ws, out, stream=None):
    _need(lut, torch.float32, "lut")
    _fits(lut, _lut_bytes(N, SHM_LAYOUT_TEXEL, SHM_F32), "lut")
    _fits(out, _lut_bytes(N // 2, SHM_LAYOUT_TEXEL, SHM_F32), "out")
    return _check(lib().shm_mip_level(_ptr(lut), N, mode, _ptr(ws), ws.numel() * ws.element_size(), _ptr(out),
                                      _stream(stream)))


def shm_query_baseline(vlut, N, n_obj, dirs, q_per_obj, method, out, stream=None):
    _need(vlut, torch.float32, "vlut")
    Q = max(n_obj, 0) * max(q_per_obj, 0)
    if Q:
        _fits(vlut, n_obj * 6 * (N + 4) ** 2 * 4, "vlut")
    _fits(dirs, Q * 12, "dirs")
    _fits(out, Q * 16, "out")
    return _check(lib().shm_query_baseline(_ptr(vlut), N, n_obj, _ptr(dirs), q_per_obj, method, _ptr(out),
                                           _stream(stream)))


def shm_sh_eval(coeffs, L, n_obj, dirs, q_per_obj, out, stream=None):
    _need(coeffs, torch.float32, "coeffs")
    Q = max(n_obj, 0) * max(q_per_obj, 0)
    if Q:
        _fits(coeffs, n_obj * (L + 1) ** 2 * 4, "coeffs")
    _fits(dirs, Q * 12, "dirs")
    _fits(out, Q * 16, "out")
    return _check(lib().shm_sh_eval(_ptr(coeffs), L, n_obj, _ptr(dirs), q_per_obj, _ptr(out), _stream(stream)))


# ---------------------------------------------------------------------------
# plans (batched form)
# ---------------------------------------------------------------------------
class Plan:
    """Owns a shm_plan: the batched persistent launch over uneven objects.

    objs: sequence of (lut_offset, N, q_begin, q_count)."""

    def __init__(self, objs, dtype, layout=SHM_LAYOUT_TEXEL, stream=None):
        arr = (shm_object * len(objs))()
        for i, (off, N, qb, qc) in enumerate(objs):
            arr[i].lut_offset, arr[i].N, arr[i].reserved, arr[i].q_begin, arr[i].q_count = int(off), int(N), 0, int(qb), int(qc)
        self._arr = arr
        self.dtype, self.layout = dtype, layout
        # extents the launches access: rows of dirs/out and bytes of the LUT
        self._rows = max((int(qb) + int(qc) for (_, _, qb, qc) in objs if int(qc) > 0), default=0)
        self._lut_bytes = max((int(off) * _dbytes(dtype) + _lut_bytes(int(N), layout, dtype)
                               for (off, N, _, qc) in objs if int(qc) > 0), default=0)
        # elements of every object's LUT (the backward writes them all)
        self._lut_elems_all = max((int(off) + _lut_bytes(int(N), layout, dtype) // _dbytes(dtype)
                                   for (off, N, _, _) in objs), default=0)
        h = ctypes.c_void_p()
        _check(lib().shm_plan_create(ctypes.cast(arr, ctypes.c_void_p), len(objs), dtype, layout, _stream(stream),
                                     ctypes.byref(h)))
        self.handle = h

    def autotune(self, lut, dirs, out, cache_path=None, stream=None):
        self._fits(lut, dirs, out)
        s = shm_launch_shape()
        _check(lib().shm_plan_autotune(self.handle, _ptr(lut), _ptr(dirs), _ptr(out),
                                       cache_path.encode() if cache_path else None, _stream(stream), ctypes.byref(s)))
        return s.as_dict()

    def set_shape(self, block, qpt, tile, grid_per_cu):
        s = shm_launch_shape(block, qpt, tile, grid_per_cu)
        _check(lib().shm_plan_set_shape(self.handle, ctypes.byref(s)))

    def _fits(self, lut, dirs, out, normal=None):
        _fits(lut, self._lut_bytes, "lut")
        _fits(dirs, self._rows * 12, "dirs")
        _fits(out, self._rows * 16, "out")
        _fits(normal, self._rows * 12, "normal")

    def launch(self, lut, dirs, out, normal=None, stream=None):
        self._fits(lut, dirs, out, normal)
        _check(lib().shm_plan_launch(self.handle, _ptr(lut), _ptr(dirs), _ptr(out), _ptr(normal), _stream(stream)))

    def capture_graph(self, lut, dirs, out, normal=None, stream=None):
        self._fits(lut, dirs, out, normal)
        _check(lib().shm_plan_capture_graph(self.handle, _ptr(lut), _ptr(dirs), _ptr(out), _ptr(normal), _stream(stream)))

    def graph_launch(self, stream=None):
        _check(lib().shm_plan_graph_launch(self.handle, _stream(stream)))

    def probe(self, lut, dirs, out, seed=20063, stream=None):
        """shm_plan_probe: the launch's memory traffic without its arithmetic
        (see shm_probe.h); out[q] = (dirs[q], bits of the footprint's word sum)."""
        self._fits(lut, dirs, out)
        _check(lib().shm_plan_probe(self.handle, _ptr(lut), _ptr(dirs), _ptr(out), seed & 0xFFFFFFFF, _stream(stream)))

    def backward_sort(self, dirs, stream=None):
        """shm_plan_backward_sort: sort the plan's queries by cell (kept in
        the plan while dirs are unchanged)."""
        _fits(dirs, self._rows * 12, "dirs")
        _check(lib().shm_plan_backward_sort(self.handle, _ptr(dirs), _stream(stream)))

    def backward(self, lut, dirs, grad_out, grad_lut=None, grad_dirs=None, stream=None):
        """shm_plan_backward: dL/dLUT (FP32, the LUT's element layout) and
        dL/d dirs of every object's rows."""
        _fits(lut, self._lut_bytes, "lut")
        _fits(dirs, self._rows * 12, "dirs")
        _fits(grad_out, self._rows * 16, "grad_out")
        _fits(grad_lut, self._lut_elems_all * 4, "grad_lut")
        _fits(grad_dirs, self._rows * 12, "grad_dirs")
        for t, name in ((grad_out, "grad_out"), (grad_lut, "grad_lut"), (grad_dirs, "grad_dirs")):
            if t is not None:
                _need(t, torch.float32, name)
        _check(lib().shm_plan_backward(self.handle, _ptr(lut), _ptr(dirs), _ptr(grad_out), _ptr(grad_lut),
                                       _ptr(grad_dirs), _stream(stream)))

    @property
    def work_items(self):
        return lib().shm_plan_work_items(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().shm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# allocating helpers
# ---------------------------------------------------------------------------
def lut_n(lut, layout=SHM_LAYOUT_TEXEL):
    """Face size N of a LUT tensor [..., 6, N+2, N+2, 4] (TEXEL) or
    [..., 6, N+1, N+1, 16] (CELL)."""
    return lut.shape[-2] - (2 if layout == SHM_LAYOUT_TEXEL else 1)


def bake_sh(coeffs, N, dtype=torch.float32, stream=None):
    """coeffs [n_obj, (L+1)^2] FP32 (device) -> LUT [n_obj, 6, N+2, N+2, 4]."""
    n_obj, K = coeffs.shape
    L = int(round(K ** 0.5)) - 1
    if (L + 1) ** 2 != K:
        raise ValueError("coeffs must have (L+1)^2 columns")
    lut = torch.empty((n_obj, 6, N + 2, N + 2, 4), dtype=dtype, device=coeffs.device)
    ws = torch.empty(max(shm_bake_sh_lut_workspace(L, N), 1), dtype=torch.uint8, device=coeffs.device)
    shm_bake_sh_lut(coeffs, L, N, n_obj, _dtype_code(lut), lut, ws, stream)
    return lut


def cells_to_f16(cells, stream=None):
    """FP32 CELL LUT(s) (any shape made of whole 16-float cells) -> FP16 cells
    in the FP16 cell encoding (value differences from corner 0)."""
    _need(cells, torch.float32, "cells")
    cells = cells.contiguous()
    out = torch.empty(cells.shape, dtype=torch.float16, device=cells.device)
    _check(lib().shm_cells_to_f16(_ptr(cells), cells.numel() // 16, _ptr(out), _stream(stream)))
    return out


def to_cells(lut, stream=None):
    """TEXEL LUT [n, 6, N+2, N+2, 4] -> CELL LUT [n, 6, N+1, N+1, 16]."""
    N = lut_n(lut)
    n_obj = lut.numel() // (6 * (N + 2) * (N + 2) * 4)
    cells = torch.empty((n_obj, 6, N + 1, N + 1, 16), dtype=lut.dtype, device=lut.device)
    shm_lut_to_cells(lut, _dtype_code(lut), N, n_obj, cells, stream)
    return cells


def query(lut, dirs, q_per_obj=None, layout=SHM_LAYOUT_TEXEL, normals=False, stream=None):
    """Value + spherical gradient: lut [n_obj, 6, ...] (TEXEL or CELL),
    dirs [n_obj * q_per_obj, 3] -> out [Q, 4] (R, grad) (+ normal [Q, 3])."""
    N = lut_n(lut, layout)
    per = 6 * (N + 2) * (N + 2) * 4 if layout == SHM_LAYOUT_TEXEL else 6 * (N + 1) * (N + 1) * 16
    n_obj = lut.numel() // per
    Q = dirs.shape[0]
    if q_per_obj is None:
        q_per_obj = Q // n_obj
    if q_per_obj * n_obj != Q:
        raise ValueError("dirs must hold n_obj * q_per_obj directions")
    out = torch.empty((Q, 4), dtype=torch.float32, device=dirs.device)
    nrm = torch.empty((Q, 3), dtype=torch.float32, device=dirs.device) if normals else None
    shm_query_value_grad(lut, _dtype_code(lut), layout, N, n_obj, dirs, q_per_obj, out, nrm, stream)
    return (out, nrm) if normals else out


def mip_level(lut, naive=False, stream=None):
    """Next mip level (N -> N/2) of one FP32 TEXEL LUT [6, N+2, N+2, 4]
    (or [1, 6, ...]): derivative-consistent, or naive box filtering."""
    N = lut_n(lut)
    out = torch.empty((6, N // 2 + 2, N // 2 + 2, 4), dtype=torch.float32, device=lut.device)
    ws = torch.empty(shm_mip_level_workspace(N), dtype=torch.uint8, device=lut.device)
    shm_mip_level(lut, N, 1 if naive else 0, ws, out, stream)
    return out.reshape(lut.shape[:-4] + out.shape)


def query_baseline(vlut, dirs, method, q_per_obj=None, stream=None):
    """Comparison reconstruction from a value-only LUT [n_obj, 6, N+4, N+4]."""
    N = vlut.shape[-1] - 4
    n_obj = vlut.numel() // (6 * (N + 4) * (N + 4))
    Q = dirs.shape[0]
    q_per_obj = Q // n_obj if q_per_obj is None else q_per_obj
    out = torch.empty((Q, 4), dtype=torch.float32, device=dirs.device)
    shm_query_baseline(vlut, N, n_obj, dirs, q_per_obj, method, out, stream)
    return out


def sh_eval(coeffs, dirs, q_per_obj=None, stream=None):
    """Direct SH evaluation (no LUT): coeffs [n_obj, (L+1)^2] -> (R, grad)."""
    n_obj, K = coeffs.shape
    L = int(round(K ** 0.5)) - 1
    Q = dirs.shape[0]
    q_per_obj = Q // n_obj if q_per_obj is None else q_per_obj
    out = torch.empty((Q, 4), dtype=torch.float32, device=dirs.device)
    shm_sh_eval(coeffs, L, n_obj, dirs, q_per_obj, out, stream)
    return out


def margin_dirs(N, device="cuda", stream=None):
    d = torch.empty((6, N + 4, N + 4, 3), dtype=torch.float32, device=device)
    shm_margin_dirs(N, d, stream)
    return d


def bake_fd(samples, N, dtype=torch.float32, stream=None):
    """samples [n_obj, 6, N+4, N+4] at margin_dirs(N) -> LUT."""
    n_obj = samples.numel() // (6 * (N + 4) * (N + 4))
    lut = torch.empty((n_obj, 6, N + 2, N + 2, 4), dtype=dtype, device=samples.device)
    shm_bake_fd(samples, N, n_obj, _dtype_code(lut), lut, stream)
    return lut


def _layout_flags(lut, signed):
    """(N, flags) of one TEXEL or CELL LUT tensor (CELL: last dimension 16)."""
    cell = lut.shape[-1] == 16
    N = lut_n(lut, SHM_LAYOUT_CELL if cell else SHM_LAYOUT_TEXEL)
    return N, (SHM_SIGNED if signed else 0) | (SHM_CELL_LUT if cell else 0)


def lut_rmax(lut, signed=False, stream=None):
    """Bezier bound of r (|r| if signed) over one TEXEL or CELL LUT."""
    N, flags = _layout_flags(lut, signed)
    r = torch.empty(1, dtype=torch.float32, device=lut.device)
    shm_lut_rmax(lut, _dtype_code(lut), N, flags, r, stream)
    return r


def cell_keys(lut_N, dirs, n_obj=1, stream=None):
    Q = dirs.shape[0]
    keys = torch.empty(Q, dtype=torch.int32, device=dirs.device)
    shm_cell_keys(lut_N, n_obj, dirs, Q // n_obj, keys, stream)
    return keys


def _bound_fields(bound_map):
    if bound_map is None:
        return 0, None
    if bound_map.dtype != torch.float32 or bound_map.dim() != 3 or bound_map.shape[0] != 6 or \
            bound_map.shape[1] != bound_map.shape[2]:
        raise ValueError("bound_map must be a [6, B, B] FP32 tensor from lut_bound_map")
    return bound_map.shape[1], _ptr(bound_map)


def lut_bound_map(lut, blocks=None, signed=False, stream=None):
    """[6, blocks, blocks] FP32 block bounds of r (|r| if signed) of one
    TEXEL or CELL LUT, for the trace's empty-space skipping.  By default a
    block spans about 4 cells (N / 4 blocks per face side, at most 64)."""
    N, flags = _layout_flags(lut, signed)
    if blocks is None:
        blocks = min(SHM_MAX_BOUND_BLOCKS, max(1, N // 4))
    out = torch.empty((6, blocks, blocks), dtype=torch.float32, device=lut.device)
    _check(lib().shm_lut_bound_map(_ptr(lut), _dtype_code(lut), N, flags, blocks, _ptr(out), _stream(stream)))
    return out


def trace(lut, center, rmax, ray_o, ray_d, n_march=20, n_bisect=8, n_newton=3, normals=True, image_width=0,
          bound_map=None, stream=None):
    """Fixed-schedule trace: t, (R, grad), normal.  image_width > 0 says the
    rays are a row-major image of that width (traced in 8 x 8 tiles);
    bound_map (lut_bound_map of this LUT) skips march samples provably
    outside the surface (the same results).  lut: TEXEL or CELL (last
    dimension 16)."""
    N, flags = _layout_flags(lut, False)
    P = ray_o.shape[0]
    t = torch.empty(P, dtype=torch.float32, device=ray_o.device)
    out = torch.empty((P, 4), dtype=torch.float32, device=ray_o.device)
    nrm = torch.empty((P, 3), dtype=torch.float32, device=ray_o.device) if normals else None
    if image_width or bound_map is not None or flags:
        bb, bp = _bound_fields(bound_map)
        prm = shm_trace_params(1.0, flags, n_march, n_bisect, n_newton, 0.0, 0.0, int(image_width), bb, bp)
        shm_trace_radial_ex(lut, _dtype_code(lut), N, center, rmax, prm, ray_o, ray_d, P, t, out, nrm, None, None,
                            stream)
    else:
        shm_trace_radial(lut, _dtype_code(lut), N, center, rmax, ray_o, ray_d, P, n_march, n_bisect, n_newton, t, out,
                         nrm, stream)
    return t, out, nrm


def trace_ex(lut, center, rmax, ray_o, ray_d, scale=1.0, signed=False, px_per_unit=0.0, eps_px=0.125, n_march=20,
             n_bisect=16, n_newton=3, normals=True, image_width=0, bound_map=None, stream=None):
    """Rendered-radius trace with the adaptive bisection budget: returns
    t, (R, grad), normal, sign of r (int8), F evaluations per ray (uint8).
    lut: TEXEL or CELL (last dimension 16)."""
    N, flags = _layout_flags(lut, signed)
    P = ray_o.shape[0]
    dev = ray_o.device
    t = torch.empty(P, dtype=torch.float32, device=dev)
    out = torch.empty((P, 4), dtype=torch.float32, device=dev)
    nrm = torch.empty((P, 3), dtype=torch.float32, device=dev) if normals else None
    sgn = torch.empty(P, dtype=torch.int8, device=dev)
    ev = torch.empty(P, dtype=torch.uint8, device=dev)
    bb, bp = _bound_fields(bound_map)
    prm = shm_trace_params(float(scale), flags, n_march, n_bisect, n_newton, float(px_per_unit),
                           float(eps_px), int(image_width), bb, bp)
    shm_trace_radial_ex(lut, _dtype_code(lut), N, center, rmax, prm, ray_o, ray_d, P, t, out, nrm, sgn, ev, stream)
    return t, out, nrm, sgn, ev


def query_scaled(lut, dirs, scale=1.0, signed=False, layout=None, normals=True, stream=None):
    """Rendered-radius query of one LUT (or n_obj LUTs with equal query
    counts): (R, grad), normal, sign of r (int8)."""
    if layout is None:
        layout = SHM_LAYOUT_CELL if lut.shape[-1] == 16 else SHM_LAYOUT_TEXEL
    N = lut_n(lut, layout)
    per = 6 * (N + 2) * (N + 2) * 4 if layout == SHM_LAYOUT_TEXEL else 6 * (N + 1) * (N + 1) * 16
    n_obj = lut.numel() // per
    Q = dirs.shape[0]
    dev = dirs.device
    out = torch.empty((Q, 4), dtype=torch.float32, device=dev)
    nrm = torch.empty((Q, 3), dtype=torch.float32, device=dev) if normals else None
    sgn = torch.empty(Q, dtype=torch.int8, device=dev)
    shm_query_scaled(lut, _dtype_code(lut), layout, N, n_obj, dirs, Q // n_obj, scale, SHM_SIGNED if signed else 0, out,
                     nrm, sgn, stream)
    return out, nrm, sgn


class BackwardContext:
    """Workspace + cached sort for repeated backward passes over fixed
    directions (a fitting loop).

    check_dense=True reads back (one wait) whether the sort listed dense
    tiles (cells of more than 32 queries); if it listed none, the backward
    calls launch no dense-tile kernel.  Worth it when the context serves many
    calls."""

    def __init__(self, N, n_obj, dirs, q_per_obj, stream=None, check_dense=False):
        self.N, self.n_obj, self.q_per_obj = N, n_obj, q_per_obj
        self.dirs = dirs
        # the sort is valid for exactly these direction values
        self.dirs_version = dirs._version
        nbytes = shm_backward_workspace(N, n_obj, q_per_obj)
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dirs.device)
        shm_backward_sort(N, n_obj, dirs, q_per_obj, self.ws, stream)
        self.sort_ready = SHM_SORT_READY
        if check_dense and shm_backward_dense_tiles(N, n_obj, q_per_obj, self.ws, stream) == 0:
            self.sort_ready = SHM_SORT_READY_SPARSE

    def backward(self, lut, grad_out, want_lut=True, want_dirs=True, stream=None):
        gl = torch.empty_like(lut) if want_lut else None
        gd = torch.empty((self.dirs.shape[0], 3), dtype=torch.float32, device=lut.device) if want_dirs else None
        shm_query_backward(lut, self.N, self.n_obj, self.dirs, self.q_per_obj, grad_out.contiguous(), gl, gd, self.ws,
                           self.sort_ready, stream)
        return gl, gd


class HermiteQuery(torch.autograd.Function):
    """out = (R, grad R) of every direction; differentiable with respect to
    the FP32 TEXEL LUT and to the directions (hand-written HIP backward)."""

    @staticmethod
    def forward(ctx, lut, dirs, bctx=None):
        N = lut_n(lut)
        n_obj = lut.numel() // (6 * (N + 2) * (N + 2) * 4)
        Q = dirs.shape[0]
        if n_obj < 1 or Q % n_obj:
            raise ValueError(f"{Q} directions do not split evenly over {n_obj} objects")
        if bctx is not None:
            if (bctx.N, bctx.n_obj, bctx.q_per_obj) != (N, n_obj, Q // n_obj):
                raise ValueError("bctx was built for another LUT size or query split")
            if (bctx.dirs.data_ptr() != dirs.data_ptr() or bctx.dirs.shape != dirs.shape
                    or dirs._version != bctx.dirs_version):
                raise ValueError("bctx was sorted for other directions (or they changed since)")
        out = torch.empty((Q, 4), dtype=torch.float32, device=dirs.device)
        shm_query_value_grad(lut, SHM_F32, SHM_LAYOUT_TEXEL, N, n_obj, dirs, Q // n_obj, out)
        if bctx is None:
            bctx = BackwardContext(N, n_obj, dirs.detach(), Q // n_obj)
        ctx.bctx = bctx
        ctx.save_for_backward(lut, dirs)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        lut, dirs = ctx.saved_tensors
        gl, gd = ctx.bctx.backward(lut, grad_out.contiguous().float(), want_lut=ctx.needs_input_grad[0],
                                   want_dirs=ctx.needs_input_grad[1])
        return gl, gd, None
