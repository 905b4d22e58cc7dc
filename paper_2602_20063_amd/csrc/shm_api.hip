// C ABI of libshm: argument validation, status codes, plans (batched form).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "shm_internal.hpp"
#include "../../include/shm_probe.h"

namespace shm {

static thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }

int device_cu_count()
{
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev] = n;
    }
    return cached[dev];
}

// launchers implemented in the kernel translation units
size_t bake_workspace_bytes(int L, int N);
int launch_bake_sh(const float* coeffs, int L, int N, int64_t n_obj, int out_dtype, void* lut, void* ws,
                   hipStream_t stream);
int launch_bake_sh_noalloc(const float* coeffs, int L, int N, int64_t n_obj, int out_dtype, void* lut,
                           hipStream_t stream);
int launch_margin_dirs(int N, float* dirs, hipStream_t stream);
int launch_bake_fd(const float* samples, int N, int64_t n_obj, int out_dtype, void* lut, hipStream_t stream);
int launch_lut_rmax(const void* lut, int dtype, int N, int flags, float* rmax_out, hipStream_t stream);
size_t backward_workspace_bytes(int N, int64_t n_obj, int64_t q_per_obj);
int launch_backward_sort(int N, int64_t n_obj, const float* dirs, int64_t q_per_obj, void* ws, hipStream_t stream);
int launch_cell_keys(int N, int64_t n_obj, const float* dirs, int64_t q_per_obj, uint32_t* keys, hipStream_t stream);
int launch_backward(const float* lut, int N, int64_t n_obj, const float* dirs, int64_t q_per_obj, const float* gout,
                    float* grad_lut, float* grad_dirs, void* ws, bool skip_dense, hipStream_t stream);
const uint32_t* backward_dense_count(int N, int64_t n_obj, int64_t q_per_obj, const void* ws);
int launch_trace(const void* lut, int dtype, int N, const float* center, float rmax, float scale, int flags,
                 float px_focal, float eps_px, const float* ray_o, const float* ray_d, int64_t P, int image_width,
                 const float* bound_map, int bound_blocks, int n_march, int n_bisect, int n_newton, float* t_out,
                 float* out, float* normal, int8_t* sign, uint8_t* evals, hipStream_t stream);
int launch_bound_map(const void* lut, int dtype, int N, int flags, int blocks, float* map, hipStream_t stream);
int launch_query_scaled(const void* lut, int dtype, int layout, int N, int64_t n_obj, const float* dirs,
                        int64_t q_per_obj, float scale, int flags, float* out, float* normal, int8_t* sign,
                        hipStream_t stream);
int launch_mesh_depth(const float* verts, int64_t V, const int32_t* tris, int64_t T, const float* center,
                      const float* dirs, int64_t P, float* depth, hipStream_t stream);
size_t mip_workspace_bytes(int N);
int launch_mip_level(const float* lut, int N, int mode, float* ws, float* out, hipStream_t stream);
int launch_fit_loss_grad(const float* out, const float* dirs, const float* tr, const float* tn, int64_t Q,
                         float w_value, float* grad, hipStream_t stream);
int launch_adam(float* p, const float* g, float* m, float* v, int64_t n4, int64_t step, float lr_value,
                float lr_deriv, float b1, float b2, float eps, hipStream_t stream);
int launch_fit_forward_loss_grad(const float* lut, int N, const float* dirs, const float* tr, const float* tn,
                                 int64_t Q, float w_value, float* grad, hipStream_t stream);
int launch_count_invalid(const float* dirs, int64_t Q, unsigned long long* count, hipStream_t stream);
int launch_cells_to_f16(const float* cells, int64_t n_cells, void* cells_f16, hipStream_t stream);
int launch_gather_footprints(const void* lut, int dtype, int layout, int N, int64_t n_obj, const float* dirs,
                             int64_t q_per_obj, float* foot, hipStream_t stream);
int launch_fit_step(const float* lut_in, float* lut_out, float* m, float* v, int N, const float* dirs, const float* tr,
                    const float* tn, int64_t Q, float w_value, int64_t step, float lr_value, float lr_deriv, float b1,
                    float b2, float eps, void* ws, bool skip_dense, hipStream_t stream);

int launch_probe_gather(const void* base, int64_t region_bytes, int64_t n_regions, int64_t per_region, int req_bytes,
                        uint32_t seed, int flags, const float* dirs, float* out, hipStream_t stream);
int launch_probe_stream(const void* base, int64_t bytes, float* sink, hipStream_t stream);
int launch_probe_mfma(int waves_per_simd, int chains, int64_t iters, double* flops, float* sink, hipStream_t stream);
int launch_probe_plan(const void* lut, int dtype, int layout, const shm_object* objs_dev, const WorkItem* items_dev,
                      int64_t n_items, const XcdSplit& split, const shm_launch_shape& shape, int n_cu,
                      const float* dirs, float* out, uint32_t seed, hipStream_t stream);

static bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

// n_obj * q_per_obj (both >= 0) exceeds limit, checked without overflow
static bool product_exceeds(int64_t n_obj, int64_t q_per_obj, int64_t limit)
{
    return q_per_obj > 0 && n_obj > limit / q_per_obj;
}
static bool valid_N(int N) { return N >= 1 && N <= SHM_MAX_N; }
static bool valid_dtype(int d) { return d == SHM_F32 || d == SHM_F16; }
static bool valid_layout(int l) { return l == SHM_LAYOUT_TEXEL || l == SHM_LAYOUT_CELL; }

}  // namespace shm

using namespace shm;

// ---------------------------------------------------------------------------
// plan (batched form)
// ---------------------------------------------------------------------------
struct shm_plan {
    int dtype = 0, layout = 0, device = 0, n_cu = 256;
    std::vector<shm_object> objs;
    shm_object* d_objs = nullptr;
    WorkItem* d_items = nullptr;
    int64_t items_cap = 0, n_items = 0;
    XcdSplit split{};
    shm_launch_shape shape{256, 2, 2048, 8};
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t signature = 0;
    // one event per stream the plan's kernel was launched on, recorded after
    // its latest launch there: the work list may be rewritten once they have
    // completed
    std::vector<std::pair<hipStream_t, hipEvent_t>> launched;
    hipEvent_t t0 = nullptr, t1 = nullptr;  // autotuner timing
    // backward of the objects (shm_plan_backward_sort): host prefix arrays
    // (cell, tile, query-tile bases; kept alive for their device copy), the
    // device copy, the sort workspace and whether a sort has been issued
    std::vector<int64_t> bwd_prefix;
    int64_t* d_bwd_prefix = nullptr;
    void* bwd_ws = nullptr;
    BwdObjectsHost bwd{};
    bool bwd_ready = false, bwd_sorted = false;
};

// Smallest work-item tile a shape may have (block 64 x 1 query per thread):
// the plan's work-list capacity is sized for it, so no shape needs more.
static constexpr int64_t kMinTile = 64;

static int64_t items_for_tile(const std::vector<shm_object>& objs, int64_t tile)
{
    int64_t n = 0;
    for (const shm_object& ob : objs) n += (ob.q_count + tile - 1) / tile;
    return n;
}

// Marks a launch of the plan's kernel on `stream` (outside graph capture:
// a captured launch runs when its graph does, see shm_plan_set_shape).
static int plan_mark_launch(shm_plan* P, hipStream_t stream)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    SHM_HIP_CHECK(hipStreamIsCapturing(stream, &st));
    if (st != hipStreamCaptureStatusNone) return SHM_OK;
    hipEvent_t ev = nullptr;
    for (auto& se : P->launched)
        if (se.first == stream) ev = se.second;
    if (!ev) {
        SHM_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        P->launched.emplace_back(stream, ev);
    }
    SHM_HIP_CHECK(hipEventRecord(ev, stream));
    return SHM_OK;
}

// Host wait for every launch of the plan's kernel issued so far.
static int plan_wait_launches(shm_plan* P)
{
    for (auto& se : P->launched) SHM_HIP_CHECK(hipEventSynchronize(se.second));
    return SHM_OK;
}

static int plan_build_items(shm_plan* P)
{
    std::vector<WorkItem> items;
    const int64_t tile = P->shape.tile;
    for (size_t o = 0; o < P->objs.size(); ++o) {
        const shm_object& ob = P->objs[o];
        for (int64_t q = 0; q < ob.q_count; q += tile) {
            WorkItem w;
            w.q0 = ob.q_begin + q;
            w.obj = (int32_t)o;
            w.n = (int32_t)std::min<int64_t>(tile, ob.q_count - q);
            items.push_back(w);
        }
    }
    const int64_t n = (int64_t)items.size();
    // slice boundaries: slice s starts at the first item whose preceding
    // queries reach s/8 of the total
    int64_t total = 0;
    for (const WorkItem& w : items) total += w.n;
    XcdSplit sp{};
    int64_t before = 0;
    int s = 1;
    for (int64_t i = 0; i < n && s < 8; ++i) {
        while (s < 8 && before * 8 >= total * s) sp.b[s++] = i;
        before += items[i].n;
    }
    while (s < 8) sp.b[s++] = n;
    sp.b[8] = n;
    if (n > P->items_cap)  // cannot happen: the capacity covers the smallest tile
        return fail(SHM_ERR_INVALID_ARG, "plan: %lld work items exceed the capacity %lld", (long long)n,
                    (long long)P->items_cap);
    // launches issued earlier may still read the old list
    if (int rc = plan_wait_launches(P)) return rc;
    P->n_items = n;
    P->split = sp;
    if (n) {
        SHM_HIP_CHECK(hipMemcpyAsync(P->d_items, items.data(), (size_t)n * sizeof(WorkItem), hipMemcpyHostToDevice,
                                     P->cap_stream));
        SHM_HIP_CHECK(hipStreamSynchronize(P->cap_stream));  // `items` is a host temporary
    }
    return SHM_OK;
}

static int check_shape(const shm_launch_shape& s)
{
    if (!(s.block == 64 || s.block == 128 || s.block == 256 || s.block == 512))
        return fail(SHM_ERR_INVALID_ARG, "shape.block must be 64, 128, 256 or 512 (got %d)", s.block);
    if (!(s.qpt == 1 || s.qpt == 2 || s.qpt == 4)) return fail(SHM_ERR_INVALID_ARG, "shape.qpt must be 1, 2 or 4");
    if (s.tile <= 0 || s.tile % (s.block * s.qpt) != 0 || s.tile > (1 << 24))
        return fail(SHM_ERR_INVALID_ARG, "shape.tile must be a positive multiple of block*qpt (<= 2^24)");
    if (s.grid_per_cu < 0 || s.grid_per_cu > 32) return fail(SHM_ERR_INVALID_ARG, "shape.grid_per_cu must be 0..32");
    return SHM_OK;
}

static uint64_t fnv1a(uint64_t h, const void* p, size_t n)
{
    const unsigned char* b = reinterpret_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    return h;
}

extern "C" {

int shm_version(void) { return SHM_ABI_VERSION; }

const char* shm_last_error(void) { return g_err.c_str(); }

int64_t shm_lut_elems(int32_t N, int32_t layout)
{
    if (!valid_N(N) || !valid_layout(layout)) return 0;
    return layout == SHM_LAYOUT_CELL ? cell_elems(N) : texel_elems(N);
}

size_t shm_bake_sh_lut_workspace(int32_t L, int32_t N)
{
    if (L < 0 || L > SHM_MAX_L || !valid_N(N)) return 0;
    return bake_workspace_bytes(L, N);
}

// arguments of both SH bakes; SHM_OK with *nothing = true when there is no work
static int check_bake_args(const float* coeffs, int32_t L, int32_t N, int64_t n_obj, int32_t out_dtype,
                           const void* lut_out, bool* nothing)
{
    *nothing = false;
    if (L < 0) return fail(SHM_ERR_INVALID_ARG, "bake: L must be >= 0 (got %d)", L);
    if (L > SHM_MAX_L) return fail(SHM_ERR_UNSUPPORTED, "bake: L must be <= %d (got %d)", SHM_MAX_L, L);
    if (!valid_N(N)) return fail(SHM_ERR_INVALID_ARG, "bake: N must be 1..%d (got %d)", SHM_MAX_N, N);
    if (n_obj < 0) return fail(SHM_ERR_INVALID_ARG, "bake: n_obj must be >= 0");
    if (product_exceeds(n_obj, texel_elems(N), INT64_MAX / 8)) return fail(SHM_ERR_UNSUPPORTED, "bake: LUT too large");
    if (!valid_dtype(out_dtype)) return fail(SHM_ERR_INVALID_ARG, "bake: bad dtype %d", out_dtype);
    if (n_obj == 0) { *nothing = true; return SHM_OK; }
    if (!coeffs || !lut_out) return fail(SHM_ERR_INVALID_ARG, "bake: null pointer");
    return SHM_OK;
}

int shm_bake_sh_lut(const float* coeffs, int32_t L, int32_t N, int64_t n_obj, int32_t out_dtype, void* lut_out,
                    void* ws, size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    bool nothing = false;
    if (int rc = check_bake_args(coeffs, L, N, n_obj, out_dtype, lut_out, &nothing)) return rc;
    if (nothing) return SHM_OK;
    if (!ws || ws_bytes < bake_workspace_bytes(L, N))
        return fail(SHM_ERR_WORKSPACE, "bake: workspace of %zu bytes needed (got %zu)", bake_workspace_bytes(L, N), ws_bytes);
    return launch_bake_sh(coeffs, L, N, n_obj, out_dtype, lut_out, ws, stream);
}

int shm_bake_sh_lut_noalloc(const float* coeffs, int32_t L, int32_t N, int64_t n_obj, int32_t out_dtype,
                            void* lut_out, hipStream_t stream)
{
    clear_error();
    bool nothing = false;
    if (int rc = check_bake_args(coeffs, L, N, n_obj, out_dtype, lut_out, &nothing)) return rc;
    const size_t need = bake_workspace_bytes(L, N);
    if (need > (size_t)SHM_BAKE_NOALLOC_MAX_BYTES)
        return fail(SHM_ERR_UNSUPPORTED,
                    "bake_noalloc: the basis table for L=%d, N=%d needs %zu bytes, more than the library's %u-byte "
                    "scratch; use shm_bake_sh_lut with a workspace", L, N, need, (unsigned)SHM_BAKE_NOALLOC_MAX_BYTES);
    if (nothing) return SHM_OK;
    return launch_bake_sh_noalloc(coeffs, L, N, n_obj, out_dtype, lut_out, stream);
}

int shm_margin_dirs(int32_t N, float* dirs, hipStream_t stream)
{
    clear_error();
    if (!valid_N(N)) return fail(SHM_ERR_INVALID_ARG, "margin_dirs: N must be 1..%d", SHM_MAX_N);
    if (!dirs) return fail(SHM_ERR_INVALID_ARG, "margin_dirs: null pointer");
    return launch_margin_dirs(N, dirs, stream);
}

int shm_bake_fd(const float* samples, int32_t N, int64_t n_obj, int32_t out_dtype, void* lut_out, hipStream_t stream)
{
    clear_error();
    if (!valid_N(N)) return fail(SHM_ERR_INVALID_ARG, "bake_fd: N must be 1..%d", SHM_MAX_N);
    if (n_obj < 0 || !valid_dtype(out_dtype)) return fail(SHM_ERR_INVALID_ARG, "bake_fd: bad n_obj or dtype");
    if (product_exceeds(n_obj, texel_elems(N), INT64_MAX / 8)) return fail(SHM_ERR_UNSUPPORTED, "bake_fd: LUT too large");
    if (n_obj == 0) return SHM_OK;
    if (!samples || !lut_out) return fail(SHM_ERR_INVALID_ARG, "bake_fd: null pointer");
    if (!aligned(lut_out, out_dtype == SHM_F16 ? 8 : 16)) return fail(SHM_ERR_INVALID_ARG, "bake_fd: misaligned LUT");
    return launch_bake_fd(samples, N, n_obj, out_dtype, lut_out, stream);
}

int shm_lut_to_cells(const void* lut_texel, int32_t dtype, int32_t N, int64_t n_obj, void* lut_cell, hipStream_t stream)
{
    clear_error();
    if (!valid_N(N) || !valid_dtype(dtype) || n_obj < 0) return fail(SHM_ERR_INVALID_ARG, "lut_to_cells: bad N, dtype or n_obj");
    if (product_exceeds(n_obj, cell_elems(N), INT64_MAX / 8)) return fail(SHM_ERR_UNSUPPORTED, "lut_to_cells: LUT too large");
    if (n_obj == 0) return SHM_OK;
    if (!lut_texel || !lut_cell) return fail(SHM_ERR_INVALID_ARG, "lut_to_cells: null pointer");
    const size_t al = dtype == SHM_F16 ? 8 : 16;
    if (!aligned(lut_texel, al) || !aligned(lut_cell, al)) return fail(SHM_ERR_INVALID_ARG, "lut_to_cells: misaligned");
    return launch_lut_to_cells(lut_texel, dtype, N, n_obj, lut_cell, stream);
}

int shm_query_value_grad(const void* lut, int32_t dtype, int32_t layout, int32_t N, int64_t n_obj, const float* dirs,
                         int64_t q_per_obj, float* out, float* normal, hipStream_t stream)
{
    clear_error();
    if (!valid_dtype(dtype)) return fail(SHM_ERR_INVALID_ARG, "query: bad dtype %d", dtype);
    if (!valid_layout(layout)) return fail(SHM_ERR_INVALID_ARG, "query: bad layout %d", layout);
    if (!valid_N(N)) return fail(SHM_ERR_INVALID_ARG, "query: N must be 1..%d (got %d)", SHM_MAX_N, N);
    if (n_obj < 0 || q_per_obj < 0) return fail(SHM_ERR_INVALID_ARG, "query: negative size");
    if (product_exceeds(n_obj, q_per_obj, INT64_MAX / 16))
        return fail(SHM_ERR_UNSUPPORTED, "query: %lld x %lld queries", (long long)n_obj, (long long)q_per_obj);
    if (n_obj == 0 || q_per_obj == 0) return SHM_OK;
    if (!lut || !dirs || !out) return fail(SHM_ERR_INVALID_ARG, "query: null pointer");
    const size_t al = (dtype == SHM_F16 && layout == SHM_LAYOUT_TEXEL) ? 8 : 16;
    if (!aligned(lut, al) || !aligned(out, 16) || !aligned(dirs, 4) || (normal && !aligned(normal, 4)))
        return fail(SHM_ERR_INVALID_ARG, "query: misaligned buffer (lut %zu B, out 16 B)", al);
    return launch_query_uniform(lut, dtype, layout, N, n_obj, dirs, q_per_obj, out, normal, stream);
}

size_t shm_query_objects_workspace(int64_t n_obj) { return n_obj < 0 ? 0 : query_objects_workspace(n_obj); }

int shm_query_objects(const void* lut, int32_t dtype, int32_t layout, const shm_object* objs, int64_t n_obj,
                      const float* dirs, float* out, float* normal, void* ws, size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    if (!valid_dtype(dtype)) return fail(SHM_ERR_INVALID_ARG, "query_objects: bad dtype %d", dtype);
    if (!valid_layout(layout)) return fail(SHM_ERR_INVALID_ARG, "query_objects: bad layout %d", layout);
    if (n_obj < 0) return fail(SHM_ERR_INVALID_ARG, "query_objects: negative object count");
    if (n_obj > INT64_MAX / 64) return fail(SHM_ERR_UNSUPPORTED, "query_objects: too many objects");
    if (n_obj == 0) return SHM_OK;
    if (!lut || !objs || !dirs || !out || !ws) return fail(SHM_ERR_INVALID_ARG, "query_objects: null pointer");
    if (ws_bytes < query_objects_workspace(n_obj))
        return fail(SHM_ERR_WORKSPACE, "query_objects: workspace of %zu bytes needed (got %zu)",
                    query_objects_workspace(n_obj), ws_bytes);
    const size_t al = (dtype == SHM_F16 && layout == SHM_LAYOUT_TEXEL) ? 8 : 16;
    if (!aligned(lut, al) || !aligned(out, 16) || !aligned(dirs, 4) || (normal && !aligned(normal, 4)) ||
        !aligned(objs, 8) || !aligned(ws, 8))
        return fail(SHM_ERR_INVALID_ARG, "query_objects: misaligned buffer (lut %zu B, out 16 B, objs and ws 8 B)", al);
    return launch_query_objects(lut, dtype, layout, objs, n_obj, dirs, out, normal, ws, stream);
}

int shm_cells_to_f16(const float* cells, int64_t n_cells, void* cells_f16, hipStream_t stream)
{
    clear_error();
    if (n_cells < 0) return fail(SHM_ERR_INVALID_ARG, "cells_to_f16: negative cell count");
    if (n_cells > INT64_MAX / 64) return fail(SHM_ERR_UNSUPPORTED, "cells_to_f16: too many cells");
    if (n_cells == 0) return SHM_OK;
    if (!cells || !cells_f16) return fail(SHM_ERR_INVALID_ARG, "cells_to_f16: null pointer");
    if (!aligned(cells, 16) || !aligned(cells_f16, 8)) return fail(SHM_ERR_INVALID_ARG, "cells_to_f16: misaligned buffer");
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(cells), b0 = reinterpret_cast<uintptr_t>(cells_f16);
    if (a0 < b0 + (uintptr_t)n_cells * 32 && b0 < a0 + (uintptr_t)n_cells * 64)
        return fail(SHM_ERR_INVALID_ARG, "cells_to_f16: input and output overlap");
    return launch_cells_to_f16(cells, n_cells, cells_f16, stream);
}

int shm_gather_footprints(const void* lut, int32_t dtype, int32_t layout, int32_t N, int64_t n_obj, const float* dirs,
                          int64_t q_per_obj, float* foot, hipStream_t stream)
{
    clear_error();
    if (!valid_dtype(dtype)) return fail(SHM_ERR_INVALID_ARG, "gather_footprints: bad dtype %d", dtype);
    if (!valid_layout(layout)) return fail(SHM_ERR_INVALID_ARG, "gather_footprints: bad layout %d", layout);
    if (!valid_N(N)) return fail(SHM_ERR_INVALID_ARG, "gather_footprints: N must be 1..%d (got %d)", SHM_MAX_N, N);
    if (n_obj < 0 || q_per_obj < 0) return fail(SHM_ERR_INVALID_ARG, "gather_footprints: negative size");
    if (product_exceeds(n_obj, q_per_obj, INT64_MAX / 64))
        return fail(SHM_ERR_UNSUPPORTED, "gather_footprints: %lld x %lld queries", (long long)n_obj, (long long)q_per_obj);
    if (n_obj == 0 || q_per_obj == 0) return SHM_OK;
    if (!lut || !dirs || !foot) return fail(SHM_ERR_INVALID_ARG, "gather_footprints: null pointer");
    const size_t al = (dtype == SHM_F16 && layout == SHM_LAYOUT_TEXEL) ? 8 : 16;
    if (!aligned(lut, al) || !aligned(foot, 16) || !aligned(dirs, 4))
        return fail(SHM_ERR_INVALID_ARG, "gather_footprints: misaligned buffer (lut %zu B, foot 16 B)", al);
    return launch_gather_footprints(lut, dtype, layout, N, n_obj, dirs, q_per_obj, foot, stream);
}

// ---------------------------------------------------------------------------
int shm_plan_create(const shm_object* objs_host, int64_t n_obj, int32_t dtype, int32_t layout, hipStream_t stream,
                    shm_plan** plan_out)
{
    clear_error();
    if (!plan_out) return fail(SHM_ERR_INVALID_ARG, "plan_create: null plan_out");
    *plan_out = nullptr;
    if (n_obj < 0 || (n_obj > 0 && !objs_host)) return fail(SHM_ERR_INVALID_ARG, "plan_create: bad object list");
    if (n_obj > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "plan_create: too many objects");
    if (!valid_dtype(dtype) || !valid_layout(layout)) return fail(SHM_ERR_INVALID_ARG, "plan_create: bad dtype/layout");
    const int64_t align_elems = (dtype == SHM_F16) ? (layout == SHM_LAYOUT_CELL ? 8 : 4) : 4;
    for (int64_t o = 0; o < n_obj; ++o) {
        const shm_object& b = objs_host[o];
        if (!valid_N(b.N)) return fail(SHM_ERR_INVALID_ARG, "plan_create: object %lld has N=%d", (long long)o, b.N);
        if (b.lut_offset < 0 || b.lut_offset % align_elems)
            return fail(SHM_ERR_INVALID_ARG, "plan_create: object %lld lut_offset %lld must be >= 0 and a multiple of %lld",
                        (long long)o, (long long)b.lut_offset, (long long)align_elems);
        if (b.q_begin < 0 || b.q_count < 0) return fail(SHM_ERR_INVALID_ARG, "plan_create: object %lld bad query range", (long long)o);
    }
    int device = 0;
    SHM_HIP_CHECK(hipGetDevice(&device));
    shm_plan* P = new shm_plan();
    P->device = device;
    P->dtype = dtype;
    P->layout = layout;
    P->objs.assign(objs_host, objs_host + n_obj);
    P->n_cu = device_cu_count();
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, &dtype, sizeof dtype);
    h = fnv1a(h, &layout, sizeof layout);
    for (auto& b : P->objs) {
        h = fnv1a(h, &b.N, sizeof b.N);
        h = fnv1a(h, &b.q_count, sizeof b.q_count);
    }
    P->signature = h;
    int rc;
    if (hipMalloc(&P->d_objs, (size_t)std::max<int64_t>(n_obj, 1) * sizeof(shm_object)) != hipSuccess) {
        delete P;
        return fail(SHM_ERR_HIP, "plan_create: hipMalloc failed");
    }
    if (n_obj && (hipMemcpyAsync(P->d_objs, objs_host, (size_t)n_obj * sizeof(shm_object), hipMemcpyHostToDevice,
                                 stream) != hipSuccess ||
                  hipStreamSynchronize(stream) != hipSuccess)) {  // objs_host may be released on return
        shm_plan_destroy(P);
        return fail(SHM_ERR_HIP, "plan_create: copy of descriptors failed");
    }
    if (hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&P->t0) != hipSuccess || hipEventCreate(&P->t1) != hipSuccess) {
        shm_plan_destroy(P);
        return fail(SHM_ERR_HIP, "plan_create: stream or event creation failed");
    }
    // the work list is sized once, for the smallest tile any shape may use
    P->items_cap = std::max<int64_t>(items_for_tile(P->objs, kMinTile), 1);
    if (hipMalloc(&P->d_items, (size_t)P->items_cap * sizeof(WorkItem)) != hipSuccess) {
        P->items_cap = 0;
        shm_plan_destroy(P);
        return fail(SHM_ERR_HIP, "plan_create: hipMalloc of the work list (%lld items) failed", (long long)P->items_cap);
    }
    if ((rc = plan_build_items(P)) != SHM_OK) {
        std::string msg = g_err;
        shm_plan_destroy(P);
        return fail(rc, "%s", msg.c_str());
    }
    *plan_out = P;
    return SHM_OK;
}

// Release a plan's captured graph (best effort: the handles are dropped
// whatever the runtime answers).
static void drop_graph(shm_plan* plan)
{
    if (plan->exec) { (void)hipGraphExecDestroy(plan->exec); plan->exec = nullptr; }
    if (plan->graph) { (void)hipGraphDestroy(plan->graph); plan->graph = nullptr; }
}

int shm_plan_set_shape(shm_plan* plan, const shm_launch_shape* shape)
{
    clear_error();
    if (!plan || !shape) return fail(SHM_ERR_INVALID_ARG, "plan_set_shape: null argument");
    int rc = check_shape(*shape);
    if (rc) return rc;
    // the plan's graph, and with a new tile the work list, may still be in
    // use by launches issued earlier
    if ((rc = plan_wait_launches(plan)) != SHM_OK) return rc;
    const bool retile = shape->tile != plan->shape.tile;
    plan->shape = *shape;
    drop_graph(plan);  // captured with the previous shape
    return retile ? plan_build_items(plan) : SHM_OK;
}

int shm_plan_launch(shm_plan* plan, const void* lut, const float* dirs, float* out, float* normal, hipStream_t stream)
{
    clear_error();
    if (!plan) return fail(SHM_ERR_INVALID_ARG, "plan_launch: null plan");
    if (plan->n_items == 0) return SHM_OK;
    if (!lut || !dirs || !out) return fail(SHM_ERR_INVALID_ARG, "plan_launch: null pointer");
    const size_t al = (plan->dtype == SHM_F16 && plan->layout == SHM_LAYOUT_TEXEL) ? 8 : 16;
    if (!aligned(lut, al) || !aligned(out, 16)) return fail(SHM_ERR_INVALID_ARG, "plan_launch: misaligned buffer");
    int rc = launch_query_persistent(lut, plan->dtype, plan->layout, plan->d_objs, plan->d_items, plan->n_items,
                                     plan->split, plan->shape, plan->n_cu, dirs, out, normal, stream);
    return rc ? rc : plan_mark_launch(plan, stream);
}

static std::map<std::string, shm_launch_shape> read_cache(const char* path)
{
    std::map<std::string, shm_launch_shape> m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        // "  "<key>": [block, qpt, tile, grid_per_cu],"
        size_t a = line.find('"'), b = line.find('"', a + 1), c = line.find('['), d = line.find(']');
        if (a == std::string::npos || b == std::string::npos || c == std::string::npos || d == std::string::npos) continue;
        shm_launch_shape s;
        if (sscanf(line.c_str() + c, "[%d, %d, %d, %d]", &s.block, &s.qpt, &s.tile, &s.grid_per_cu) == 4 && check_shape(s) == SHM_OK)
            m[line.substr(a + 1, b - a - 1)] = s;
    }
    clear_error();
    return m;
}

static void write_cache(const char* path, const std::map<std::string, shm_launch_shape>& m)
{
    std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        f << "{\n";
        size_t i = 0;
        for (auto& kv : m) {
            f << "  \"" << kv.first << "\": [" << kv.second.block << ", " << kv.second.qpt << ", " << kv.second.tile
              << ", " << kv.second.grid_per_cu << "]" << (++i < m.size() ? "," : "") << "\n";
        }
        f << "}\n";
    }
    std::rename(tmp.c_str(), path);
}

int shm_plan_autotune(shm_plan* plan, const void* lut, const float* dirs, float* out, const char* cache_path,
                      hipStream_t stream, shm_launch_shape* chosen)
{
    clear_error();
    if (!plan || !lut || !dirs || !out) return fail(SHM_ERR_INVALID_ARG, "plan_autotune: null argument");
    char key[96];
    {
        hipDeviceProp_t prop;
        SHM_HIP_CHECK(hipGetDeviceProperties(&prop, plan->device));
        snprintf(key, sizeof key, "%s/%d/%016llx", prop.gcnArchName, plan->n_cu, (unsigned long long)plan->signature);
        for (char* c = key; *c; ++c)
            if (*c == '"' || *c == '\\') *c = '_';
    }
    std::map<std::string, shm_launch_shape> cache;
    if (cache_path) {
        cache = read_cache(cache_path);
        auto it = cache.find(key);
        if (it != cache.end()) {
            int rc = shm_plan_set_shape(plan, &it->second);
            if (rc) return rc;
            if (chosen) *chosen = it->second;
            return SHM_OK;
        }
    }
    std::vector<shm_launch_shape> cands;
    for (int block : {256, 512})
        for (int qpt : {1, 2, 4})
            for (int mult : {1, 4, 16})
                for (int gpc : {0, 4, 8, 16})  // 0: one workgroup per work item
                    if (gpc > 0 || mult < 16) cands.push_back(shm_launch_shape{block, qpt, block * qpt * mult, gpc});
    hipEvent_t e0 = plan->t0, e1 = plan->t1;
    float best_ms = 1e30f;
    shm_launch_shape best = plan->shape;
    int rc = SHM_OK;
    for (const auto& s : cands) {
        if ((rc = shm_plan_set_shape(plan, &s)) != SHM_OK) break;
        if ((rc = shm_plan_launch(plan, lut, dirs, out, nullptr, stream)) != SHM_OK) break;  // warm-up
        if (hipEventRecord(e0, stream) != hipSuccess) { rc = fail(SHM_ERR_HIP, "plan_autotune: event record failed"); break; }
        const int reps = 3;
        for (int r = 0; r < reps && rc == SHM_OK; ++r) rc = shm_plan_launch(plan, lut, dirs, out, nullptr, stream);
        if (rc) break;
        if (hipEventRecord(e1, stream) != hipSuccess) { rc = fail(SHM_ERR_HIP, "plan_autotune: event record failed"); break; }
        if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(SHM_ERR_HIP, "plan_autotune: event sync failed"); break; }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = fail(SHM_ERR_HIP, "plan_autotune: elapsed time failed"); break; }
        ms /= reps;
        if (ms < best_ms) { best_ms = ms; best = s; }
    }
    if (rc) return rc;
    if ((rc = shm_plan_set_shape(plan, &best)) != SHM_OK) return rc;
    if (chosen) *chosen = best;
    if (cache_path) {
        cache[key] = best;
        write_cache(cache_path, cache);
    }
    return SHM_OK;
}

int shm_plan_capture_graph(shm_plan* plan, const void* lut, const float* dirs, float* out, float* normal, hipStream_t stream)
{
    clear_error();
    if (!plan) return fail(SHM_ERR_INVALID_ARG, "plan_capture_graph: null plan");
    (void)stream;
    if (int rc0 = plan_wait_launches(plan)) return rc0;  // a replay of the old graph may still run
    drop_graph(plan);
    SHM_HIP_CHECK(hipStreamSynchronize(plan->cap_stream));
    SHM_HIP_CHECK(hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = shm_plan_launch(plan, lut, dirs, out, normal, plan->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(plan->cap_stream, &g);
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (e != hipSuccess) return fail(SHM_ERR_HIP, "plan_capture_graph: end capture: %s", hipGetErrorString(e));
    plan->graph = g;
    e = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        plan->graph = nullptr;
        plan->exec = nullptr;
        return fail(SHM_ERR_HIP, "plan_capture_graph: instantiate: %s", hipGetErrorString(e));
    }
    return SHM_OK;
}

int shm_plan_graph_launch(shm_plan* plan, hipStream_t stream)
{
    clear_error();
    if (!plan || !plan->exec) return fail(SHM_ERR_INVALID_ARG, "plan_graph_launch: no captured graph");
    SHM_HIP_CHECK(hipGraphLaunch(plan->exec, stream));
    return plan_mark_launch(plan, stream);
}

int64_t shm_plan_work_items(const shm_plan* plan) { return plan ? plan->n_items : -1; }

int shm_plan_destroy(shm_plan* plan)
{
    if (!plan) return SHM_OK;
    // best-effort cleanup: every resource is released even if one call fails;
    // launches still in flight finish first
    (void)plan_wait_launches(plan);
    clear_error();
    drop_graph(plan);
    for (auto& se : plan->launched) (void)hipEventDestroy(se.second);
    if (plan->t0) (void)hipEventDestroy(plan->t0);
    if (plan->t1) (void)hipEventDestroy(plan->t1);
    if (plan->cap_stream) {
        (void)hipStreamSynchronize(plan->cap_stream);
        (void)hipStreamDestroy(plan->cap_stream);
    }
    if (plan->d_items) (void)hipFree(plan->d_items);
    if (plan->d_objs) (void)hipFree(plan->d_objs);
    if (plan->d_bwd_prefix) (void)hipFree(plan->d_bwd_prefix);
    if (plan->bwd_ws) (void)hipFree(plan->bwd_ws);
    delete plan;
    return SHM_OK;
}

// Host side of a plan's backward: checks that the objects' LUTs and query
// ranges do not overlap, builds the prefix arrays and allocates the device
// copy and the sort workspace (once per plan).
static int plan_backward_prepare(shm_plan* P, hipStream_t stream)
{
    if (P->bwd_ready) return SHM_OK;
    if (P->layout != SHM_LAYOUT_TEXEL)
        return fail(SHM_ERR_UNSUPPORTED, "plan_backward: the backward takes TEXEL LUTs (the gradient is per texel)");
    const int64_t n = (int64_t)P->objs.size();
    // LUT extents [off, off + texel_elems) and query ranges must not overlap
    std::vector<std::pair<int64_t, int64_t>> lut_r, q_r;
    for (const shm_object& o : P->objs) {
        lut_r.emplace_back(o.lut_offset, o.lut_offset + texel_elems(o.N));
        if (o.q_count > 0) q_r.emplace_back(o.q_begin, o.q_begin + o.q_count);
    }
    std::sort(lut_r.begin(), lut_r.end());
    std::sort(q_r.begin(), q_r.end());
    for (size_t i = 1; i < lut_r.size(); ++i)
        if (lut_r[i].first < lut_r[i - 1].second)
            return fail(SHM_ERR_INVALID_ARG, "plan_backward: two objects' LUTs overlap (each texel has one gradient)");
    for (size_t i = 1; i < q_r.size(); ++i)
        if (q_r[i].first < q_r[i - 1].second)
            return fail(SHM_ERR_INVALID_ARG, "plan_backward: two objects' query ranges overlap");
    const int64_t BT = backward_tile_texels(), QT = backward_query_tile();
    std::vector<int64_t> pre(3 * (size_t)(n + 1));
    int64_t* cb = pre.data();
    int64_t* tb = cb + (n + 1);
    int64_t* qb = tb + (n + 1);
    int64_t Q = 0;
    for (int64_t o = 0; o < n; ++o) {
        const shm_object& ob = P->objs[o];
        const int64_t C = ob.N + 1, tpf = (ob.N + 2 + BT - 1) / BT;
        cb[o + 1] = cb[o] + 6 * C * C;
        tb[o + 1] = tb[o] + 6 * tpf * tpf;
        qb[o + 1] = qb[o] + (ob.q_count + QT - 1) / QT;
        if (ob.q_count > 0) Q = std::max(Q, ob.q_begin + ob.q_count);
    }
    // 32-bit sort keys (the key n_cells marks an invalid direction) and
    // query indices; one-dimensional grids
    if (cb[n] >= 0xffffffffll || Q >= 0xffffffffll || tb[n] > 0x7fffffff || qb[n] > 0x7fffffff)
        return fail(SHM_ERR_UNSUPPORTED, "plan_backward: %lld cells, %lld queries exceed the 32-bit sort",
                    (long long)cb[n], (long long)Q);
    BwdObjectsHost H;
    H.n_obj = n;
    H.Q = Q;
    H.n_cells = cb[n];
    H.n_tiles = tb[n];
    H.n_qtiles = qb[n];
    // the object of every tile and query tile (int32), after the prefixes
    const size_t n64 = pre.size();
    pre.resize(n64 + (size_t)((tb[n] + qb[n] + 1) / 2));
    cb = pre.data();
    tb = cb + (n + 1);
    qb = tb + (n + 1);
    int32_t* t_obj = reinterpret_cast<int32_t*>(pre.data() + n64);
    int32_t* q_obj = t_obj + tb[n];
    for (int64_t o = 0; o < n; ++o) {
        for (int64_t t = tb[o]; t < tb[o + 1]; ++t) t_obj[t] = (int32_t)o;
        for (int64_t t = qb[o]; t < qb[o + 1]; ++t) q_obj[t] = (int32_t)o;
    }
    const size_t ws_bytes = backward_objects_workspace_bytes(Q, H.n_cells, H.n_tiles);
    if (hipMalloc(&P->d_bwd_prefix, pre.size() * sizeof(int64_t)) != hipSuccess) {
        P->d_bwd_prefix = nullptr;
        return fail(SHM_ERR_HIP, "plan_backward: hipMalloc of the object prefixes failed");
    }
    if (hipMalloc(&P->bwd_ws, std::max<size_t>(ws_bytes, 256)) != hipSuccess) {
        P->bwd_ws = nullptr;
        (void)hipFree(P->d_bwd_prefix);
        P->d_bwd_prefix = nullptr;
        return fail(SHM_ERR_HIP, "plan_backward: hipMalloc of %zu bytes of sort workspace failed", ws_bytes);
    }
    P->bwd_prefix = std::move(pre);
    SHM_HIP_CHECK(hipMemcpyAsync(P->d_bwd_prefix, P->bwd_prefix.data(), P->bwd_prefix.size() * sizeof(int64_t),
                                 hipMemcpyHostToDevice, stream));
    H.objs = P->d_objs;
    H.cell_base = P->d_bwd_prefix;
    H.tile_base = P->d_bwd_prefix + (n + 1);
    H.qtile_base = P->d_bwd_prefix + 2 * (n + 1);
    H.tile_obj = reinterpret_cast<const int32_t*>(P->d_bwd_prefix + n64);
    H.qtile_obj = H.tile_obj + H.n_tiles;
    P->bwd = H;
    P->bwd_ready = true;
    return SHM_OK;
}

int shm_plan_backward_sort(shm_plan* plan, const float* dirs, hipStream_t stream)
{
    clear_error();
    if (!plan) return fail(SHM_ERR_INVALID_ARG, "plan_backward_sort: null plan");
    int rc = plan_backward_prepare(plan, stream);
    if (rc) return rc;
    if (plan->bwd.Q > 0 && (!dirs || !aligned(dirs, 4)))
        return fail(SHM_ERR_INVALID_ARG, "plan_backward_sort: null or misaligned dirs");
    // an earlier backward may still read the sort this call rewrites: the
    // stream orders it if it ran on the same stream; else wait for it
    if ((rc = plan_wait_launches(plan)) != SHM_OK) return rc;
    rc = launch_backward_sort_objects(plan->bwd, dirs, plan->bwd_ws, stream);
    if (rc) return rc;
    // how many dense tiles the sort listed: the backward launches their
    // kernel only when there are some, with a grid to match
    plan->bwd.n_dense = 0;
    if (plan->bwd.Q > 0 && plan->bwd.n_tiles > 0) {
        uint32_t n_dense = 0;
        SHM_HIP_CHECK(hipMemcpyAsync(&n_dense, backward_objects_dense_count(plan->bwd, plan->bwd_ws), sizeof n_dense,
                                     hipMemcpyDeviceToHost, stream));
        SHM_HIP_CHECK(hipStreamSynchronize(stream));
        plan->bwd.n_dense = n_dense;
    }
    plan->bwd_sorted = true;
    return plan_mark_launch(plan, stream);
}

int shm_plan_backward(shm_plan* plan, const void* lut, const float* dirs, const float* grad_out, float* grad_lut,
                      float* grad_dirs, hipStream_t stream)
{
    clear_error();
    if (!plan) return fail(SHM_ERR_INVALID_ARG, "plan_backward: null plan");
    if (!plan->bwd_sorted) return fail(SHM_ERR_INVALID_ARG, "plan_backward: call shm_plan_backward_sort first");
    if (!grad_lut && !grad_dirs) return SHM_OK;
    const BwdObjectsHost& H = plan->bwd;
    if (H.Q > 0 && (!dirs || !grad_out)) return fail(SHM_ERR_INVALID_ARG, "plan_backward: null dirs or grad_out");
    if (grad_dirs && H.Q > 0 && !lut) return fail(SHM_ERR_INVALID_ARG, "plan_backward: null lut");
    const size_t al = plan->dtype == SHM_F16 ? 8 : 16;
    if ((lut && !aligned(lut, al)) || (grad_out && !aligned(grad_out, 16)) || (grad_lut && !aligned(grad_lut, 16)) ||
        (dirs && !aligned(dirs, 4)) || (grad_dirs && !aligned(grad_dirs, 4)))
        return fail(SHM_ERR_INVALID_ARG, "plan_backward: misaligned buffer");
    int rc = launch_backward_objects(H, plan->dtype, lut, dirs, grad_out, grad_lut, grad_dirs, plan->bwd_ws, stream);
    return rc ? rc : plan_mark_launch(plan, stream);
}

// ---------------------------------------------------------------------------
size_t shm_backward_workspace(int32_t N, int64_t n_obj, int64_t q_per_obj)
{
    if (!valid_N(N) || n_obj < 0 || q_per_obj < 0 || n_obj > 0xffffffffll || product_exceeds(n_obj, q_per_obj, 0xfffffffell))
        return 0;
    return backward_workspace_bytes(N, n_obj, q_per_obj);
}

static int check_bwd(int32_t N, int64_t n_obj, int64_t q_per_obj, const void* ws, size_t ws_bytes)
{
    if (!valid_N(N)) return fail(SHM_ERR_INVALID_ARG, "backward: N must be 1..%d", SHM_MAX_N);
    if (n_obj < 0 || q_per_obj < 0) return fail(SHM_ERR_INVALID_ARG, "backward: negative size");
    if (n_obj > 0xffffffffll || product_exceeds(n_obj, q_per_obj, 0xfffffffell))
        return fail(SHM_ERR_UNSUPPORTED, "backward: more than 2^32 queries or cells");
    const int64_t Q = n_obj * q_per_obj;  // < 2^32: no overflow
    const int64_t cells = n_obj * 6ll * (N + 1) * (N + 1);
    if (Q >= 0xffffffffll || cells + 1 >= 0xffffffffll)
        return fail(SHM_ERR_UNSUPPORTED, "backward: more than 2^32 queries or cells");
    if (!ws || ws_bytes < backward_workspace_bytes(N, n_obj, q_per_obj))
        return fail(SHM_ERR_WORKSPACE, "backward: workspace of %zu bytes needed (got %zu)",
                    backward_workspace_bytes(N, n_obj, q_per_obj), ws_bytes);
    if (!aligned(ws, 256)) return fail(SHM_ERR_INVALID_ARG, "backward: workspace must be 256-byte aligned");
    return SHM_OK;
}

int shm_backward_sort(int32_t N, int64_t n_obj, const float* dirs, int64_t q_per_obj, void* ws, size_t ws_bytes,
                      hipStream_t stream)
{
    clear_error();
    int rc = check_bwd(N, n_obj, q_per_obj, ws, ws_bytes);
    if (rc) return rc;
    if (n_obj * q_per_obj > 0 && !dirs) return fail(SHM_ERR_INVALID_ARG, "backward_sort: null dirs");
    return launch_backward_sort(N, n_obj, dirs, q_per_obj, ws, stream);
}

int shm_cell_keys(int32_t N, int64_t n_obj, const float* dirs, int64_t q_per_obj, uint32_t* keys, hipStream_t stream)
{
    clear_error();
    if (!valid_N(N) || n_obj < 0 || q_per_obj < 0) return fail(SHM_ERR_INVALID_ARG, "cell_keys: bad N or size");
    if (n_obj > 0xffffffffll || n_obj * 6ll * (N + 1) * (N + 1) >= 0xffffffffll || product_exceeds(n_obj, q_per_obj, INT64_MAX / 16))
        return fail(SHM_ERR_UNSUPPORTED, "cell_keys: more than 2^32 cells or too many queries");
    if (n_obj * q_per_obj == 0) return SHM_OK;
    if (!dirs || !keys) return fail(SHM_ERR_INVALID_ARG, "cell_keys: null pointer");
    return launch_cell_keys(N, n_obj, dirs, q_per_obj, keys, stream);
}

int shm_query_backward(const float* lut, int32_t N, int64_t n_obj, const float* dirs, int64_t q_per_obj,
                       const float* grad_out, float* grad_lut, float* grad_dirs, void* ws, size_t ws_bytes,
                       int32_t sort_ready, hipStream_t stream)
{
    clear_error();
    int rc = check_bwd(N, n_obj, q_per_obj, ws, ws_bytes);
    if (rc) return rc;
    const int64_t Q = n_obj * q_per_obj;
    if (!lut && (grad_dirs || grad_lut)) return fail(SHM_ERR_INVALID_ARG, "backward: null lut");
    if (Q > 0 && (!dirs || !grad_out)) return fail(SHM_ERR_INVALID_ARG, "backward: null dirs or grad_out");
    if (!aligned(lut, 16) || (grad_lut && !aligned(grad_lut, 16)) || (grad_out && !aligned(grad_out, 16)))
        return fail(SHM_ERR_INVALID_ARG, "backward: lut, grad_lut and grad_out must be 16-byte aligned");
    if (sort_ready < 0 || sort_ready > SHM_SORT_READY_SPARSE)
        return fail(SHM_ERR_INVALID_ARG, "backward: sort_ready must be 0, SHM_SORT_READY or SHM_SORT_READY_SPARSE");
    if (!sort_ready && (rc = launch_backward_sort(N, n_obj, dirs, q_per_obj, ws, stream)) != SHM_OK) return rc;
    return launch_backward(lut, N, n_obj, dirs, q_per_obj, grad_out, grad_lut, grad_dirs, ws,
                           sort_ready == SHM_SORT_READY_SPARSE, stream);
}

int64_t shm_backward_dense_tiles(int32_t N, int64_t n_obj, int64_t q_per_obj, const void* ws, size_t ws_bytes,
                                 hipStream_t stream)
{
    clear_error();
    if (check_bwd(N, n_obj, q_per_obj, ws, ws_bytes) != SHM_OK) return -1;
    if (n_obj * q_per_obj == 0) return 0;  // the sort lists nothing without queries
    uint32_t count = 0;
    hipError_t e = hipMemcpyAsync(&count, backward_dense_count(N, n_obj, q_per_obj, ws), sizeof(count),
                                  hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        fail(SHM_ERR_HIP, "backward_dense_tiles: %s", hipGetErrorString(e));
        return -1;
    }
    return (int64_t)count;
}

// ---------------------------------------------------------------------------
static int check_trace_params(const shm_trace_params* tp)
{
    if (!tp) return fail(SHM_ERR_INVALID_ARG, "trace: null params");
    if (!(tp->scale > 0.0f) || !std::isfinite(tp->scale)) return fail(SHM_ERR_INVALID_ARG, "trace: scale must be positive and finite");
    if (tp->flags & ~(SHM_SIGNED | SHM_CELL_LUT)) return fail(SHM_ERR_INVALID_ARG, "trace: unknown flags 0x%x", tp->flags);
    if (tp->n_march < 1 || tp->n_bisect < 0 || tp->n_newton < 0 || tp->n_march + tp->n_bisect + tp->n_newton + 1 > 64)
        return fail(SHM_ERR_INVALID_ARG, "trace: iteration counts must satisfy n_march >= 1 and total <= 64");
    if (!std::isfinite(tp->px_per_unit) || tp->px_per_unit < 0.0f)
        return fail(SHM_ERR_INVALID_ARG, "trace: px_per_unit must be finite and >= 0");
    if (tp->px_per_unit > 0.0f && !(tp->eps_px > 0.0f && std::isfinite(tp->eps_px)))
        return fail(SHM_ERR_INVALID_ARG, "trace: eps_px must be positive and finite with an adaptive budget");
    if (tp->image_width < 0) return fail(SHM_ERR_INVALID_ARG, "trace: negative image_width");
    if (tp->bound_blocks < 0 || tp->bound_blocks > SHM_MAX_BOUND_BLOCKS)
        return fail(SHM_ERR_INVALID_ARG, "trace: bound_blocks must be 0..%d", SHM_MAX_BOUND_BLOCKS);
    if (tp->bound_blocks > 0 && (!tp->bound_map || !aligned(tp->bound_map, 4)))
        return fail(SHM_ERR_INVALID_ARG, "trace: bound_blocks > 0 needs a bound map");
    return SHM_OK;
}

int shm_trace_radial_ex(const void* lut, int32_t dtype, int32_t N, const float* center, float rmax,
                        const shm_trace_params* params, const float* ray_o, const float* ray_d, int64_t P, float* t_out,
                        float* out, float* normal, int8_t* sign, uint8_t* evals, hipStream_t stream)
{
    clear_error();
    if (!valid_dtype(dtype) || !valid_N(N)) return fail(SHM_ERR_INVALID_ARG, "trace: bad dtype or N");
    if (P < 0) return fail(SHM_ERR_INVALID_ARG, "trace: negative ray count");
    if (!(rmax > 0.0f) || !std::isfinite(rmax)) return fail(SHM_ERR_INVALID_ARG, "trace: rmax must be positive and finite");
    int rc = check_trace_params(params);
    if (rc) return rc;
    if (!center) return fail(SHM_ERR_INVALID_ARG, "trace: null center");
    if (params->image_width > 0 && P % params->image_width != 0)
        return fail(SHM_ERR_INVALID_ARG, "trace: %lld rays are not whole rows of width %d", (long long)P,
                    params->image_width);
    if (P == 0) return SHM_OK;
    if (!lut || !ray_o || !ray_d || !t_out || !out) return fail(SHM_ERR_INVALID_ARG, "trace: null pointer");
    const size_t al = (dtype == SHM_F16 && !(params->flags & SHM_CELL_LUT)) ? 8 : 16;
    if (!aligned(lut, al) || !aligned(out, 16)) return fail(SHM_ERR_INVALID_ARG, "trace: misaligned buffer");
    return launch_trace(lut, dtype, N, center, rmax, params->scale, params->flags, params->px_per_unit, params->eps_px,
                        ray_o, ray_d, P, params->image_width, params->bound_map, params->bound_blocks,
                        params->n_march, params->n_bisect, params->n_newton, t_out, out, normal, sign, evals, stream);
}

int shm_trace_radial(const void* lut, int32_t dtype, int32_t N, const float* center, float rmax, const float* ray_o,
                     const float* ray_d, int64_t P, int32_t n_march, int32_t n_bisect, int32_t n_newton, float* t_out,
                     float* out, float* normal, hipStream_t stream)
{
    const shm_trace_params tp = {1.0f, 0, n_march, n_bisect, n_newton, 0.0f, 0.0f, 0, 0, nullptr};
    return shm_trace_radial_ex(lut, dtype, N, center, rmax, &tp, ray_o, ray_d, P, t_out, out, normal, nullptr, nullptr,
                               stream);
}

int shm_lut_bound_map(const void* lut, int32_t dtype, int32_t N, int32_t flags, int32_t blocks, float* map_out,
                      hipStream_t stream)
{
    clear_error();
    if (!valid_dtype(dtype) || !valid_N(N)) return fail(SHM_ERR_INVALID_ARG, "bound_map: bad dtype or N");
    if (flags & ~(SHM_SIGNED | SHM_CELL_LUT)) return fail(SHM_ERR_INVALID_ARG, "bound_map: unknown flags 0x%x", flags);
    if (blocks < 1 || blocks > SHM_MAX_BOUND_BLOCKS)
        return fail(SHM_ERR_INVALID_ARG, "bound_map: blocks must be 1..%d", SHM_MAX_BOUND_BLOCKS);
    if (!lut || !map_out) return fail(SHM_ERR_INVALID_ARG, "bound_map: null pointer");
    if (!aligned(map_out, 4) || !aligned(lut, (flags & SHM_CELL_LUT) ? 16 : (dtype == SHM_F16 ? 2 : 4)))
        return fail(SHM_ERR_INVALID_ARG, "bound_map: misaligned buffer");
    return launch_bound_map(lut, dtype, N, flags, blocks, map_out, stream);
}

int shm_lut_rmax(const void* lut, int32_t dtype, int32_t N, int32_t flags, float* rmax_out, hipStream_t stream)
{
    clear_error();
    if (!valid_dtype(dtype) || !valid_N(N)) return fail(SHM_ERR_INVALID_ARG, "lut_rmax: bad dtype or N");
    if (flags & ~(SHM_SIGNED | SHM_CELL_LUT)) return fail(SHM_ERR_INVALID_ARG, "lut_rmax: unknown flags 0x%x", flags);
    if (!lut || !rmax_out) return fail(SHM_ERR_INVALID_ARG, "lut_rmax: null pointer");
    if (!aligned(rmax_out, 4) || ((flags & SHM_CELL_LUT) && !aligned(lut, 16)))
        return fail(SHM_ERR_INVALID_ARG, "lut_rmax: misaligned buffer");
    return launch_lut_rmax(lut, dtype, N, flags, rmax_out, stream);
}

int shm_query_scaled(const void* lut, int32_t dtype, int32_t layout, int32_t N, int64_t n_obj, const float* dirs,
                     int64_t q_per_obj, float scale, int32_t flags, float* out, float* normal, int8_t* sign,
                     hipStream_t stream)
{
    clear_error();
    if (!valid_dtype(dtype) || !valid_layout(layout) || !valid_N(N))
        return fail(SHM_ERR_INVALID_ARG, "query_scaled: bad dtype, layout or N");
    if (n_obj < 0 || q_per_obj < 0) return fail(SHM_ERR_INVALID_ARG, "query_scaled: negative size");
    if (product_exceeds(n_obj, q_per_obj, INT64_MAX / 16)) return fail(SHM_ERR_UNSUPPORTED, "query_scaled: too many queries");
    if (!(scale > 0.0f) || !std::isfinite(scale)) return fail(SHM_ERR_INVALID_ARG, "query_scaled: scale must be positive and finite");
    if (flags & ~SHM_SIGNED) return fail(SHM_ERR_INVALID_ARG, "query_scaled: unknown flags 0x%x", flags);
    if (n_obj * q_per_obj == 0) return SHM_OK;
    if (!lut || !dirs || !out) return fail(SHM_ERR_INVALID_ARG, "query_scaled: null pointer");
    const size_t al = (dtype == SHM_F16 && layout == SHM_LAYOUT_TEXEL) ? 8 : 16;
    if (!aligned(lut, al) || !aligned(out, 16) || !aligned(dirs, 4) || (normal && !aligned(normal, 4)))
        return fail(SHM_ERR_INVALID_ARG, "query_scaled: misaligned buffer (lut %zu B, out 16 B)", al);
    return launch_query_scaled(lut, dtype, layout, N, n_obj, dirs, q_per_obj, scale, flags, out, normal, sign, stream);
}

int shm_mesh_radial_depth(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                          const float* center, const float* dirs, int64_t P, float* depth, hipStream_t stream)
{
    clear_error();
    if (n_verts < 0 || n_tris < 0 || P < 0) return fail(SHM_ERR_INVALID_ARG, "mesh_depth: negative size");
    if (n_verts > 0x7fffffffll) return fail(SHM_ERR_UNSUPPORTED, "mesh_depth: more than 2^31 - 1 vertices");
    if (!center) return fail(SHM_ERR_INVALID_ARG, "mesh_depth: null center");
    if (!std::isfinite(center[0]) || !std::isfinite(center[1]) || !std::isfinite(center[2]))
        return fail(SHM_ERR_INVALID_ARG, "mesh_depth: center must be finite");
    if (P == 0) return SHM_OK;
    if (!dirs || !depth) return fail(SHM_ERR_INVALID_ARG, "mesh_depth: null dirs or depth");
    if (n_tris > 0 && (!tris || !verts)) return fail(SHM_ERR_INVALID_ARG, "mesh_depth: null mesh");
    if (!aligned(depth, 4) || !aligned(dirs, 4) || (tris && !aligned(tris, 4)) || (verts && !aligned(verts, 4)))
        return fail(SHM_ERR_INVALID_ARG, "mesh_depth: misaligned buffer");
    return launch_mesh_depth(verts, n_verts, tris, n_tris, center, dirs, P, depth, stream);
}

// ---------------------------------------------------------------------------
int shm_fit_loss_grad(const float* out, const float* dirs, const float* target_r, const float* target_n, int64_t Q,
                      float w_value, float* grad, hipStream_t stream)
{
    clear_error();
    if (Q < 0) return fail(SHM_ERR_INVALID_ARG, "fit_loss_grad: negative query count");
    if (!std::isfinite(w_value) || w_value < 0.0f) return fail(SHM_ERR_INVALID_ARG, "fit_loss_grad: w_value must be finite and >= 0");
    if (Q == 0) return SHM_OK;
    if (!out || !dirs || !target_r || !target_n || !grad) return fail(SHM_ERR_INVALID_ARG, "fit_loss_grad: null pointer");
    if (!aligned(out, 16) || !aligned(grad, 16) || !aligned(dirs, 4) || !aligned(target_r, 4) || !aligned(target_n, 4))
        return fail(SHM_ERR_INVALID_ARG, "fit_loss_grad: misaligned buffer (out and grad need 16 bytes)");
    return launch_fit_loss_grad(out, dirs, target_r, target_n, Q, w_value, grad, stream);
}

int shm_fit_forward_loss_grad(const float* lut, int32_t N, const float* dirs, const float* target_r,
                              const float* target_n, int64_t Q, float w_value, float* grad, hipStream_t stream)
{
    clear_error();
    if (!valid_N(N)) return fail(SHM_ERR_INVALID_ARG, "fit_forward_loss_grad: bad N");
    if (Q < 0) return fail(SHM_ERR_INVALID_ARG, "fit_forward_loss_grad: negative query count");
    if (!std::isfinite(w_value) || w_value < 0.0f)
        return fail(SHM_ERR_INVALID_ARG, "fit_forward_loss_grad: w_value must be finite and >= 0");
    if (Q == 0) return SHM_OK;
    if (!lut || !dirs || !target_r || !target_n || !grad) return fail(SHM_ERR_INVALID_ARG, "fit_forward_loss_grad: null pointer");
    if (!aligned(lut, 16) || !aligned(grad, 16) || !aligned(dirs, 4) || !aligned(target_r, 4) || !aligned(target_n, 4))
        return fail(SHM_ERR_INVALID_ARG, "fit_forward_loss_grad: misaligned buffer (lut and grad need 16 bytes)");
    return launch_fit_forward_loss_grad(lut, N, dirs, target_r, target_n, Q, w_value, grad, stream);
}

int shm_adam_step(float* param, const float* grad, float* m, float* v, int64_t n4, int64_t step, float lr_value,
                  float lr_deriv, float beta1, float beta2, float eps, hipStream_t stream)
{
    clear_error();
    if (n4 < 0 || step < 1) return fail(SHM_ERR_INVALID_ARG, "adam: need n4 >= 0 and step >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) || !std::isfinite(eps) ||
        !std::isfinite(lr_value) || !std::isfinite(lr_deriv))
        return fail(SHM_ERR_INVALID_ARG, "adam: need 0 <= beta < 1, finite eps > 0 and finite learning rates");
    if (n4 == 0) return SHM_OK;
    if (!param || !grad || !m || !v) return fail(SHM_ERR_INVALID_ARG, "adam: null pointer");
    if (!aligned(param, 16) || !aligned(grad, 16) || !aligned(m, 16) || !aligned(v, 16))
        return fail(SHM_ERR_INVALID_ARG, "adam: buffers must be 16-byte aligned");
    return launch_adam(param, grad, m, v, n4, step, lr_value, lr_deriv, beta1, beta2, eps, stream);
}

int shm_count_invalid(const float* dirs, int64_t Q, unsigned long long* count, hipStream_t stream)
{
    clear_error();
    if (Q < 0) return fail(SHM_ERR_INVALID_ARG, "count_invalid: negative query count");
    if (Q > INT64_MAX / 12) return fail(SHM_ERR_UNSUPPORTED, "count_invalid: too many queries");
    if (!count || !aligned(count, 8)) return fail(SHM_ERR_INVALID_ARG, "count_invalid: count must be an 8-byte aligned device pointer");
    if (Q > 0 && (!dirs || !aligned(dirs, 4))) return fail(SHM_ERR_INVALID_ARG, "count_invalid: null or misaligned dirs");
    return launch_count_invalid(dirs, Q, count, stream);
}

static bool ranges_overlap(const void* a, const void* b, size_t bytes)
{
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bytes && y < x + bytes;
}

int shm_fit_step(const float* lut_in, float* lut_out, float* m, float* v, int32_t N, const float* dirs,
                 const float* target_r, const float* target_n, int64_t Q, float w_value, int64_t step, float lr_value,
                 float lr_deriv, float beta1, float beta2, float eps, void* ws, size_t ws_bytes, int32_t sort_ready,
                 hipStream_t stream)
{
    clear_error();
    int rc = check_bwd(N, 1, Q, ws, ws_bytes);
    if (rc) return rc;
    if (!std::isfinite(w_value) || w_value < 0.0f)
        return fail(SHM_ERR_INVALID_ARG, "fit_step: w_value must be finite and >= 0");
    if (step < 1) return fail(SHM_ERR_INVALID_ARG, "fit_step: step must be >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f) || !std::isfinite(eps) ||
        !std::isfinite(lr_value) || !std::isfinite(lr_deriv))
        return fail(SHM_ERR_INVALID_ARG, "fit_step: need 0 <= beta < 1, finite eps > 0 and finite learning rates");
    if (!lut_in || !lut_out || !m || !v) return fail(SHM_ERR_INVALID_ARG, "fit_step: null LUT or moment buffer");
    if (Q > 0 && (!dirs || !target_r || !target_n)) return fail(SHM_ERR_INVALID_ARG, "fit_step: null dirs or targets");
    if (!aligned(lut_in, 16) || !aligned(lut_out, 16) || !aligned(m, 16) || !aligned(v, 16) ||
        (Q > 0 && (!aligned(dirs, 4) || !aligned(target_r, 4) || !aligned(target_n, 4))))
        return fail(SHM_ERR_INVALID_ARG, "fit_step: misaligned buffer (LUTs and moments need 16 bytes)");
    const size_t bytes = (size_t)texel_elems(N) * sizeof(float);
    const void* bufs[4] = {lut_in, lut_out, m, v};
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j)
            if (ranges_overlap(bufs[i], bufs[j], bytes))
                return fail(SHM_ERR_INVALID_ARG, "fit_step: lut_in, lut_out, m and v must not overlap");
    if (sort_ready < 0 || sort_ready > SHM_SORT_READY_SPARSE)
        return fail(SHM_ERR_INVALID_ARG, "fit_step: sort_ready must be 0, SHM_SORT_READY or SHM_SORT_READY_SPARSE");
    if (!sort_ready && Q > 0 && (rc = launch_backward_sort(N, 1, dirs, Q, ws, stream)) != SHM_OK) return rc;
    return launch_fit_step(lut_in, lut_out, m, v, N, dirs, target_r, target_n, Q, w_value, step, lr_value, lr_deriv,
                           beta1, beta2, eps, ws, sort_ready == SHM_SORT_READY_SPARSE, stream);
}

// ---------------------------------------------------------------------------
size_t shm_mip_level_workspace(int32_t N)
{
    if (!valid_N(N) || N < 2 || (N & 1)) return 0;
    return mip_workspace_bytes(N);
}

int shm_mip_level(const float* lut, int32_t N, int32_t mode, void* ws, size_t ws_bytes, float* out, hipStream_t stream)
{
    clear_error();
    if (!valid_N(N) || N < 2 || (N & 1)) return fail(SHM_ERR_INVALID_ARG, "mip_level: N must be even, 2..%d", SHM_MAX_N);
    if (mode != 0 && mode != 1) return fail(SHM_ERR_INVALID_ARG, "mip_level: mode must be 0 or 1");
    if (!lut || !out) return fail(SHM_ERR_INVALID_ARG, "mip_level: null pointer");
    if (!aligned(lut, 16) || !aligned(out, 16)) return fail(SHM_ERR_INVALID_ARG, "mip_level: misaligned LUT");
    if (!ws || ws_bytes < mip_workspace_bytes(N))
        return fail(SHM_ERR_WORKSPACE, "mip_level: workspace of %zu bytes needed (got %zu)", mip_workspace_bytes(N), ws_bytes);
    return launch_mip_level(lut, N, mode, reinterpret_cast<float*>(ws), out, stream);
}

// ---------------------------------------------------------------------------
int shm_query_baseline(const float* vlut, int32_t N, int64_t n_obj, const float* dirs, int64_t q_per_obj,
                       int32_t method, float* out, hipStream_t stream)
{
    clear_error();
    if (!valid_N(N)) return fail(SHM_ERR_INVALID_ARG, "query_baseline: N must be 1..%d", SHM_MAX_N);
    if (method < SHM_RECON_NEAREST || method > SHM_RECON_FAST_BICUBIC_FD) return fail(SHM_ERR_INVALID_ARG, "query_baseline: bad method %d", method);
    if (n_obj < 0 || q_per_obj < 0) return fail(SHM_ERR_INVALID_ARG, "query_baseline: negative size");
    if (product_exceeds(n_obj, q_per_obj, INT64_MAX / 16)) return fail(SHM_ERR_UNSUPPORTED, "query_baseline: too many queries");
    if (n_obj == 0 || q_per_obj == 0) return SHM_OK;
    if (!vlut || !dirs || !out) return fail(SHM_ERR_INVALID_ARG, "query_baseline: null pointer");
    if (!aligned(out, 16) || !aligned(vlut, 4) || !aligned(dirs, 4)) return fail(SHM_ERR_INVALID_ARG, "query_baseline: misaligned buffer");
    return launch_query_baseline(vlut, N, n_obj, dirs, q_per_obj, method, out, stream);
}

int shm_sh_eval(const float* coeffs, int32_t L, int64_t n_obj, const float* dirs, int64_t q_per_obj, float* out,
                hipStream_t stream)
{
    clear_error();
    if (L < 0) return fail(SHM_ERR_INVALID_ARG, "sh_eval: L must be >= 0");
    if (L > SHM_MAX_L) return fail(SHM_ERR_UNSUPPORTED, "sh_eval: L must be <= %d", SHM_MAX_L);
    if (n_obj < 0 || q_per_obj < 0) return fail(SHM_ERR_INVALID_ARG, "sh_eval: negative size");
    if (product_exceeds(n_obj, q_per_obj, INT64_MAX / 16)) return fail(SHM_ERR_UNSUPPORTED, "sh_eval: too many queries");
    if (n_obj == 0 || q_per_obj == 0) return SHM_OK;
    if (!coeffs || !dirs || !out) return fail(SHM_ERR_INVALID_ARG, "sh_eval: null pointer");
    if (!aligned(out, 16)) return fail(SHM_ERR_INVALID_ARG, "sh_eval: misaligned output");
    return launch_sh_eval(coeffs, L, n_obj, dirs, q_per_obj, out, stream);
}


// ---------------------------------------------------------------------------
// memory-system probes
// ---------------------------------------------------------------------------
int shm_probe_gather(const void* base, int64_t region_bytes, int64_t n_regions, int64_t per_region, int32_t req_bytes,
                     uint32_t seed, int32_t flags, const float* dirs, float* out, hipStream_t stream)
{
    clear_error();
    if (!(req_bytes == 0 || req_bytes == 16 || req_bytes == 32 || req_bytes == 64 || req_bytes == 128))
        return fail(SHM_ERR_INVALID_ARG, "probe_gather: req_bytes must be 0, 16, 32, 64 or 128 (got %d)", req_bytes);
    if (flags & ~(SHM_PROBE_DIRS | SHM_PROBE_OUT)) return fail(SHM_ERR_INVALID_ARG, "probe_gather: unknown flags %d", flags);
    if (n_regions < 0 || per_region < 0) return fail(SHM_ERR_INVALID_ARG, "probe_gather: negative size");
    if (region_bytes < req_bytes || region_bytes < 16 || region_bytes % 16)
        return fail(SHM_ERR_INVALID_ARG, "probe_gather: region_bytes must be a multiple of 16 and >= req_bytes");
    if (req_bytes && region_bytes / req_bytes > 0xffffffffll)
        return fail(SHM_ERR_UNSUPPORTED, "probe_gather: region too large");
    if (product_exceeds(n_regions, region_bytes, INT64_MAX / 2) || product_exceeds(n_regions, per_region, INT64_MAX / 16))
        return fail(SHM_ERR_UNSUPPORTED, "probe_gather: sizes overflow");
    const int64_t tiles = (per_region + 255) / 256;
    if (product_exceeds(n_regions, tiles, 0x7fffffff)) return fail(SHM_ERR_UNSUPPORTED, "probe_gather: grid too large");
    if (n_regions == 0 || per_region == 0) return SHM_OK;
    if ((req_bytes && !base) || !out || ((flags & SHM_PROBE_DIRS) && !dirs))
        return fail(SHM_ERR_INVALID_ARG, "probe_gather: null pointer");
    if ((req_bytes && !aligned(base, 16)) || !aligned(out, 16) || (dirs && !aligned(dirs, 4)))
        return fail(SHM_ERR_INVALID_ARG, "probe_gather: misaligned buffer");
    return launch_probe_gather(base, region_bytes, n_regions, per_region, req_bytes, seed, flags,
                               (flags & SHM_PROBE_DIRS) ? dirs : nullptr, out, stream);
}

int shm_probe_stream_read(const void* base, int64_t bytes, float* sink, hipStream_t stream)
{
    clear_error();
    if (bytes < 0 || bytes % 16) return fail(SHM_ERR_INVALID_ARG, "probe_stream_read: bytes must be a multiple of 16");
    if (bytes == 0) return SHM_OK;
    if (!base || !sink) return fail(SHM_ERR_INVALID_ARG, "probe_stream_read: null pointer");
    if (!aligned(base, 16) || !aligned(sink, 16)) return fail(SHM_ERR_INVALID_ARG, "probe_stream_read: misaligned buffer");
    return launch_probe_stream(base, bytes, sink, stream);
}

int shm_probe_mfma_f32(int32_t waves_per_simd, int32_t chains, int64_t iters, double* flops, float* sink,
                       hipStream_t stream)
{
    clear_error();
    if (waves_per_simd < 1 || waves_per_simd > 8) return fail(SHM_ERR_INVALID_ARG, "probe_mfma: waves_per_simd must be 1..8");
    if (chains != 1 && chains != 2 && chains != 4 && chains != 8)
        return fail(SHM_ERR_INVALID_ARG, "probe_mfma: chains must be 1, 2, 4 or 8");
    if (iters < 1) return fail(SHM_ERR_INVALID_ARG, "probe_mfma: iters must be >= 1");
    if (!flops || !sink) return fail(SHM_ERR_INVALID_ARG, "probe_mfma: null pointer");
    if (!aligned(sink, 16)) return fail(SHM_ERR_INVALID_ARG, "probe_mfma: misaligned sink");
    return launch_probe_mfma(waves_per_simd, chains, iters, flops, sink, stream);
}

int shm_plan_probe(shm_plan* plan, const void* lut, const float* dirs, float* out, uint32_t seed, hipStream_t stream)
{
    clear_error();
    if (!plan) return fail(SHM_ERR_INVALID_ARG, "plan_probe: null plan");
    if (plan->n_items == 0) return SHM_OK;
    if (!lut || !dirs || !out) return fail(SHM_ERR_INVALID_ARG, "plan_probe: null pointer");
    const size_t al = (plan->dtype == SHM_F16 && plan->layout == SHM_LAYOUT_TEXEL) ? 8 : 16;
    if (!aligned(lut, al) || !aligned(out, 16)) return fail(SHM_ERR_INVALID_ARG, "plan_probe: misaligned buffer");
    int rc = launch_probe_plan(lut, plan->dtype, plan->layout, plan->d_objs, plan->d_items, plan->n_items, plan->split,
                               plan->shape, plan->n_cu, dirs, out, seed, stream);
    return rc ? rc : plan_mark_launch(plan, stream);
}

}  // extern "C"
