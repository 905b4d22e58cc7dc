// Host-side internals shared by the translation units of libshm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/shm.h"

namespace shm {

// thread-local last-error message; returns `code` for convenient chaining
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define SHM_HIP_CHECK(expr)                                                                   \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return ::shm::fail(SHM_ERR_HIP, "%s: %s (%s:%d)", #expr,        \
                                                 hipGetErrorString(e_), __FILE__, __LINE__);  \
    } while (0)

#define SHM_LAUNCH_CHECK()                                                                    \
    do {                                                                                      \
        hipError_t e_ = hipGetLastError();                                                    \
        if (e_ != hipSuccess) return ::shm::fail(SHM_ERR_HIP, "kernel launch: %s (%s:%d)",    \
                                                 hipGetErrorString(e_), __FILE__, __LINE__);  \
    } while (0)

inline int64_t texel_elems(int N) { return 6ll * (N + 2) * (N + 2) * 4; }
inline int64_t cell_elems(int N) { return 6ll * (N + 1) * (N + 1) * 16; }
inline size_t dtype_bytes(int dt) { return dt == SHM_F16 ? 2 : 4; }

// number of compute units of the current device (cached per device)
int device_cu_count();

// work item of the persistent query kernel: queries [q0, q0 + n) of object obj
struct WorkItem {
    int64_t q0;
    int32_t obj;
    int32_t n;
};

// The work list cut into 8 contiguous slices of (nearly) equal query counts,
// slice s = items [b[s], b[s+1]): the blocks of one XCD (blockIdx % 8 under
// round-robin dispatch) walk one slice, so an object's items share one L2.
struct XcdSplit {
    int64_t b[9];
};

// Grid of a plan launch.  grid_per_cu > 0: a persistent grid of that many
// workgroups per CU (at most one per item).  grid_per_cu 0: one workgroup
// per work item; the slices hold (nearly) equal query counts, not item
// counts, so each XCD gets as many workgroups as the largest slice has items
// and none walks a second item (those of smaller slices exit at once).
inline int64_t plan_grid(const shm_launch_shape& shape, int n_cu, int64_t n_items, const XcdSplit& split)
{
    int64_t G;
    if (shape.grid_per_cu == 0 && n_items >= 8) {
        int64_t most = 0;
        for (int s = 0; s < 8; ++s) most = split.b[s + 1] - split.b[s] > most ? split.b[s + 1] - split.b[s] : most;
        G = 8 * most;
    } else {
        G = shape.grid_per_cu == 0 ? n_items : (int64_t)shape.grid_per_cu * n_cu;
        if (G > n_items) G = n_items;
    }
    return G > 0x7fffffff ? 0x7fffffff : G;
}

// device copy of a host shm_object (same layout)
static_assert(sizeof(shm_object) == 32, "shm_object layout");

// launchers (validated arguments)
int launch_query_uniform(const void* lut, int dtype, int layout, int N, int64_t n_obj, const float* dirs,
                         int64_t q_per_obj, float* out, float* normal, hipStream_t stream);
int launch_query_persistent(const void* lut, int dtype, int layout, const shm_object* objs_dev,
                            const WorkItem* items_dev, int64_t n_items, const XcdSplit& split,
                            const shm_launch_shape& shape, int n_cu,
                            const float* dirs, float* out, float* normal, hipStream_t stream);
// backward of a plan's objects: device prefix arrays (n_obj + 1 entries each)
// and the totals the host derived from the descriptors
struct BwdObjectsHost {
    const shm_object* objs = nullptr;
    const int64_t* cell_base = nullptr;
    const int64_t* tile_base = nullptr;
    const int64_t* qtile_base = nullptr;
    const int32_t* tile_obj = nullptr;   // object of each LUT-gradient tile
    const int32_t* qtile_obj = nullptr;  // object of each query tile
    int64_t n_obj = 0, Q = 0, n_cells = 0, n_tiles = 0, n_qtiles = 0;
    int64_t n_dense = 0;  // dense tiles found by the last sort (read back by the plan)
};
int backward_tile_texels();   // texels per side of a LUT-gradient tile
int backward_query_tile();    // queries per query tile of the object kernels
size_t backward_objects_workspace_bytes(int64_t Q, int64_t n_cells, int64_t n_tiles);
const uint32_t* backward_objects_dense_count(const BwdObjectsHost& H, const void* ws);  // device address
int launch_backward_sort_objects(const BwdObjectsHost& H, const float* dirs, void* ws, hipStream_t stream);
int launch_backward_objects(const BwdObjectsHost& H, int dtype, const void* lut, const float* dirs, const float* gout,
                            float* grad_lut, float* grad_dirs, void* ws, hipStream_t stream);
size_t query_objects_workspace(int64_t n_obj);
int launch_query_objects(const void* lut, int dtype, int layout, const shm_object* objs, int64_t n_obj,
                         const float* dirs, float* out, float* normal, void* ws, hipStream_t stream);
int launch_lut_to_cells(const void* lut, int dtype, int N, int64_t n_obj, void* cells, hipStream_t stream);
int launch_query_baseline(const float* vlut, int N, int64_t n_obj, const float* dirs, int64_t q_per_obj, int method,
                          float* out, hipStream_t stream);
int launch_sh_eval(const float* coeffs, int L, int64_t n_obj, const float* dirs, int64_t q_per_obj, float* out,
                   hipStream_t stream);

}  // namespace shm
