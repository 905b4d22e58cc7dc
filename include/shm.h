/*
 * shm.h -- C ABI of the MI355X (gfx950) Spherical Hermite Maps library.
 *
 * Spherical Hermite Maps (Abouagour & Garyfallidis, arXiv 2602.20063) store a
 * star-shaped radial function R(w) in a padded cube map whose texels hold the
 * value and scaled chart derivatives (r, r_u h, r_v h, r_uv h^2), h = 1/N
 * (Sec. 3.3, Eq. 2).  A query maps a direction to a face and (u, v), gathers
 * one 2x2 texel footprint (16 scalars) and applies bicubic Hermite
 * reconstruction (Eqs. 3-5); the chart derivatives become the spherical
 * gradient through the cube-map metric tensor (Sec. 3.4, Eqs. 6-9) and the
 * normal follows from Eq. 10.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers unless the comment says "host".
 *    The caller allocates and owns every buffer, including workspaces; the
 *    library never frees caller memory.  It allocates device memory only in
 *    shm_plan_create and in a plan's first shm_plan_backward_sort (both
 *    released by shm_plan_destroy).
 *  - Every call is asynchronous on the given HIP stream (0 = the null
 *    stream); arguments are validated on the host before anything is
 *    enqueued.  The exceptions are the plan calls that say they wait
 *    (shm_plan_create, shm_plan_set_shape, shm_plan_autotune,
 *    shm_plan_capture_graph, shm_plan_backward_sort, shm_plan_destroy):
 *    each blocks the host until
 *    its own copies, or the plan's earlier launches, have completed; none
 *    waits for the whole device.  Calls return SHM_OK or an error code and
 *    never throw; shm_last_error() gives a thread-local message for the last
 *    failure (every entry point that validates arguments clears it first).
 *  - Faces are ordered +X, -X, +Y, -Y, +Z, -Z with the hardware cube-map
 *    (s, t) orientation: d/|ma| = M + sc S + tc T, u = (sc+1)/2,
 *    v = (tc+1)/2 (Sec. 3.2).  Face ties go X before Y before Z, and a
 *    component >= 0 (including -0) selects the positive face.
 *  - TEXEL layout (the paper's padded cube map, Sec. 3.2-3.3):
 *      lut[obj][face][q][p][ch], q = v row 0..N+1, p = u column 0..N+1,
 *      ch = (r, r_u h, r_v h, r_uv h^2); padded texel p has its centre at
 *      u = (p - 1/2)/N, p = 0 and N+1 are the one-texel gutter.
 *    CELL layout (derived copy of the same data for the gather): every cell
 *      (i0, j0), i0, j0 in 0..N, stores its whole 2x2 footprint contiguously:
 *      lut[obj][face][j0][i0][corner][ch], corner = (i0,j0), (i0+1,j0),
 *      (i0,j0+1), (i0+1,j0+1), so one query reads one aligned 64 B (FP32)
 *      or 32 B (FP16) block.  In FP16 cells corners 1..3 hold r as its
 *      difference from corner 0's r (the other channels as they are): the
 *      patch's derivatives do not see the rounding of r itself, so FP16
 *      cells made from FP32 data (shm_cells_to_f16) keep FP16's relative
 *      precision in the gradient.  Make FP16 cells with shm_lut_to_cells or
 *      shm_cells_to_f16, not by an elementwise cast.
 *  - Queries: directions need not be unit length (w = d/|d|).  A zero or
 *    non-finite direction is not an error: its outputs are NaN.
 *  - Output of a query: out[q] = (R, gx, gy, gz) with (gx, gy, gz) the
 *    spherical gradient of R as an ambient vector (tangent to the sphere);
 *    normal[q] = (R w - grad R) / |R w - grad R| (Eq. 10), optional.
 */
#ifndef SHM_H
#define SHM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHM_ABI_VERSION 1

#if defined(__GNUC__)
#define SHM_API __attribute__((visibility("default")))
#else
#define SHM_API
#endif

typedef enum {
    SHM_OK = 0,
    SHM_ERR_INVALID_ARG = 1, /* null pointer, size out of range, bad enum */
    SHM_ERR_UNSUPPORTED = 2, /* valid but not implemented (e.g. L > 16)  */
    SHM_ERR_WORKSPACE = 3,   /* workspace missing or too small            */
    SHM_ERR_HIP = 4          /* a HIP runtime call failed                 */
} shm_status;

typedef enum { SHM_F32 = 0, SHM_F16 = 1 } shm_dtype;
typedef enum { SHM_LAYOUT_TEXEL = 0, SHM_LAYOUT_CELL = 1 } shm_layout;

#define SHM_MAX_N 1024 /* largest interior face resolution */
#define SHM_MAX_L 16   /* largest SH order of the analytic bake */
#define SHM_MAX_BOUND_BLOCKS 64 /* largest blocks per face side of a bound map */

/* ABI version (SHM_ABI_VERSION). */
SHM_API int shm_version(void);

/* Message of the last failed call on this thread ("" if none).  The pointer
 * stays valid until the next call on this thread. */
SHM_API const char* shm_last_error(void);

/* Number of scalar elements of one object's LUT: 6 (N+2)^2 4 for TEXEL,
 * 6 (N+1)^2 16 for CELL.  0 for an invalid N or layout. */
SHM_API int64_t shm_lut_elems(int32_t N, int32_t layout);

/* ------------------------------------------------------------------------
 * Bake, analytic SH mode (Sec. 3.3 Alg. 1; "Analytic SH derivatives").
 * Every padded texel, gutter included, gets (G, G_u h, G_v h, G_uv h^2) of
 * G(u,v) = sum_k coeffs[k] Y_k(normalise(M + (2u-1) S + (2v-1) T)), with
 * orthonormal real SH (no Condon-Shortley phase), k = l^2 + l + m.
 *   coeffs   [n_obj][(L+1)^2] FP32 (any affine map already folded in)
 *   L        0..16;  N 1..SHM_MAX_N;  n_obj >= 1
 *   lut_out  [n_obj][6][N+2][N+2][4] in out_dtype (TEXEL layout)
 *   ws       workspace of shm_bake_sh_lut_workspace(L, N) bytes: the SH
 *            basis table (value, h-scaled first and mixed derivatives at
 *            every padded texel), rebuilt by every call
 * The contraction coeffs x basis runs on the matrix cores (FP32 MFMA, FP32
 * accumulation); the basis table is evaluated in FP64 and stored in FP32.
 * The l = 0 term is not part of the contraction: Y_00 is constant, so it
 * adds coeffs[0] Y_00 (formed in FP64, rounded once) to every value texel
 * and nothing to the derivative channels, once, after the l >= 1 sum.
 * ---------------------------------------------------------------------- */
SHM_API size_t shm_bake_sh_lut_workspace(int32_t L, int32_t N);
SHM_API int shm_bake_sh_lut(const float* coeffs, int32_t L, int32_t N, int64_t n_obj, int32_t out_dtype, void* lut_out,
                    void* ws, size_t ws_bytes, hipStream_t stream);

/* The same bake for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no workspace argument and no allocation; the basis table lives in a
 * scratch array of SHM_BAKE_NOALLOC_MAX_BYTES inside the library (one per
 * device, held until the process ends).  Bits identical to shm_bake_sh_lut.
 * Returns SHM_ERR_UNSUPPORTED when shm_bake_sh_lut_workspace(L, N) exceeds
 * that size (L <= 16 fits up to N = 32, L <= 8 up to N = 62).  Every call on
 * a device shares its array: calls that overlap on one device (different
 * streams, no ordering between them) race and must not be issued. */
#define SHM_BAKE_NOALLOC_MAX_BYTES (32u << 20)
SHM_API int shm_bake_sh_lut_noalloc(const float* coeffs, int32_t L, int32_t N, int64_t n_obj, int32_t out_dtype,
                                    void* lut_out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Bake, general mode (Sec. 3.3 Alg. 1 with central differences and a
 * one-texel bake-time margin).
 * shm_margin_dirs writes the unit directions at which the caller samples its
 * function: dirs [6][N+4][N+4][3] FP32, index p in 0..N+3 at u=(p-3/2)/N
 * (p = 1..N+2 are the stored texels 0..N+1, p = 0 and N+3 the margin).
 * shm_bake_fd turns samples [n_obj][6][N+4][N+4] FP32 taken at those
 * directions into LUTs [n_obj][6][N+2][N+2][4] (TEXEL, out_dtype):
 *   r_u h = (r[p+1] - r[p-1]) / 2,  r_v h likewise,
 *   r_uv h^2 = (r[p+1,q+1] - r[p+1,q-1] - r[p-1,q+1] + r[p-1,q-1]) / 4.
 * ---------------------------------------------------------------------- */
SHM_API int shm_margin_dirs(int32_t N, float* dirs, hipStream_t stream);
SHM_API int shm_bake_fd(const float* samples, int32_t N, int64_t n_obj, int32_t out_dtype, void* lut_out, hipStream_t stream);

/* TEXEL -> CELL copy of n_obj LUTs of face size N (same dtype; FP16 cells
 * in the FP16 cell encoding above, the differences formed exactly in FP32
 * and rounded once). */
SHM_API int shm_lut_to_cells(const void* lut_texel, int32_t dtype, int32_t N, int64_t n_obj, void* lut_cell,
                     hipStream_t stream);
/* FP32 CELL data -> FP16 cells in the FP16 cell encoding: n_cells whole
 * cells (16 floats each, any face sizes back to back; cells 16-byte and
 * cells_f16 8-byte aligned, not overlapping); each difference is formed in
 * FP32 and rounded once, every other channel rounded once. */
SHM_API int shm_cells_to_f16(const float* cells, int64_t n_cells, void* cells_f16, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Query, value + gradient (Sec. 3.2-3.4, Eqs. 3-10): the hot path.
 * n_obj objects of one face size N, stored back to back in `lut`
 * (shm_lut_elems(N, layout) elements each); object o answers the queries
 * dirs[o*q_per_obj .. (o+1)*q_per_obj).
 *   lut     FP32 or FP16 (dtype), TEXEL or CELL (layout); FP16 data are
 *           decoded to FP32 and all arithmetic is FP32
 *   dirs    [n_obj*q_per_obj][3] FP32
 *   out     [n_obj*q_per_obj][4] FP32 (R, gx, gy, gz)
 *   normal  [n_obj*q_per_obj][3] FP32 or NULL
 * The face and cell are decided in FP32 by: a = sc/ma, u = (a+1)*0.5,
 * f = u*N + 0.5, i0 = min(floor(f), N), every step correctly rounded.  The
 * face is the exact one; the cell is the exact one (floor of the exact f)
 * except where f lies within a few FP32 ulps of an integer, where it may be
 * the neighbouring cell: the patch is C1 across cell edges, so value and
 * gradient agree there to rounding.
 * ---------------------------------------------------------------------- */
SHM_API int shm_query_value_grad(const void* lut, int32_t dtype, int32_t layout, int32_t N, int64_t n_obj, const float* dirs,
                         int64_t q_per_obj, float* out, float* normal, hipStream_t stream);

/* Step a3 of the query alone (Sec. 3.2): the 2x2 footprint of every query,
 * decided and loaded exactly as shm_query_value_grad does (same arguments),
 * written as foot [n_obj*q_per_obj][4][4] FP32 (16-byte aligned): corners
 * (i0,j0), (i0+1,j0), (i0,j0+1), (i0+1,j0+1), each (r, r_u h, r_v h,
 * r_uv h^2), FP16 data decoded; NaN for an invalid direction.  For custom
 * reconstructions, and as the gather-only cost of the query. */
SHM_API int shm_gather_footprints(const void* lut, int32_t dtype, int32_t layout, int32_t N, int64_t n_obj,
                                  const float* dirs, int64_t q_per_obj, float* foot, hipStream_t stream);

/* Counter of bad queries: adds to *count (one device uint64, zeroed by the
 * caller) the number of the Q directions dirs[Q][3] that every query entry
 * point answers with NaN: a zero vector or a NaN or Inf component.  The
 * directions need not be unit length (any nonzero finite vector is valid).
 * Integer atomics only (one per wavefront); no memset, so it may be
 * captured in a graph beside the query. */
SHM_API int shm_count_invalid(const float* dirs, int64_t Q, unsigned long long* count, hipStream_t stream);

/* Query of the rendered radius (Sec. 3.1) for a user scale s > 0:
 * R = s r for a nonnegative function; with SHM_SIGNED, R = s |r| and
 * grad R = s sign(r) grad r (chain rule of Sec. 3.4, after Eq. 10; sign(0)
 * = 0), so the normal of Eq. 10 stays outward on negative lobes.
 *   out [Q][4] (R, grad R), normal [Q][3] or NULL, sign [Q] int8 (+1, -1,
 *   0; 0 also for an invalid direction) or NULL.
 * Other arguments and the cell decision as in shm_query_value_grad. */
#define SHM_SIGNED 1
/* Flag of shm_trace_radial_ex (shm_trace_params.flags), shm_lut_rmax and
 * shm_lut_bound_map: the LUT is in the CELL layout (16-byte aligned), read
 * as a query reads it (FP16 cells decoded). */
#define SHM_CELL_LUT 2
SHM_API int shm_query_scaled(const void* lut, int32_t dtype, int32_t layout, int32_t N, int64_t n_obj, const float* dirs,
                             int64_t q_per_obj, float scale, int32_t flags, float* out, float* normal, int8_t* sign,
                             hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched form: many objects of different face sizes and query counts in
 * one persistent launch.  Objects are described on the HOST:
 *   lut_offset  element offset of the object's LUT inside `lut`
 *   N           face size 1..SHM_MAX_N
 *   q_begin     first query of the object in dirs/out
 *   q_count     number of queries (>= 0)
 * A plan owns the device copy of the descriptors, the work list (object,
 * query range) items, the chosen launch shape and optionally a captured HIP
 * graph.  The LUT dtype/layout are fixed at creation.
 * ---------------------------------------------------------------------- */
typedef struct shm_object {
    int64_t lut_offset;
    int32_t N;
    int32_t reserved;
    int64_t q_begin;
    int64_t q_count;
} shm_object;

typedef struct shm_plan shm_plan;

/* Query of objects described in DEVICE memory, without a plan (the object
 * form of the value + gradient query, Sec. 3.2-3.4): objs [n_obj]
 * shm_object on the device (8-byte aligned); object o answers the queries
 * dirs[q_begin .. q_begin + q_count) from its LUT at lut + lut_offset
 * elements (face size N) in the given dtype and layout, writing out (and
 * normal, if not NULL) at the same rows, bit for bit as shm_query_value_grad
 * answers them.  The ranges may come in any order and must not overlap.
 * The descriptors are read on the device only: an object with N outside
 * 1..SHM_MAX_N, a negative or misaligned lut_offset (a multiple of 8
 * elements for FP16 cells, else 4), a negative q_begin or q_count <= 0 is
 * skipped (its rows are not written); the caller guarantees that every
 * answered object's LUT and rows lie inside the buffers.  Two launches on
 * `stream` (a one-workgroup scan of the objects' tile counts into ws, then a
 * persistent grid over all tiles, a contiguous slice per XCD); no host
 * synchronisation, no allocation, capturable in a graph.
 *   ws  shm_query_objects_workspace(n_obj) bytes, 8-byte aligned (n_obj + 1
 *       int64 tile offsets), overwritten.
 * Errors: SHM_ERR_INVALID_ARG (bad dtype/layout, negative n_obj, null or
 * misaligned pointer), SHM_ERR_WORKSPACE (ws too small). */
SHM_API size_t shm_query_objects_workspace(int64_t n_obj);
SHM_API int shm_query_objects(const void* lut, int32_t dtype, int32_t layout, const shm_object* objs, int64_t n_obj,
                              const float* dirs, float* out, float* normal, void* ws, size_t ws_bytes,
                              hipStream_t stream);

/* Launch shape of the plan's kernel.  With qpt 2 or 4 a thread issues the
 * loads of all its queries before their arithmetic (same results as qpt 1).
 * grid_per_cu 0 launches 8 x (items of the largest of the 8 per-XCD
 * slices of the work list) workgroups, so that none takes a second item. */
typedef struct shm_launch_shape {
    int32_t block;       /* threads per workgroup: 64, 128, 256 or 512        */
    int32_t qpt;         /* queries per thread per pass: 1, 2 or 4            */
    int32_t tile;        /* queries per work item, a multiple of block * qpt  */
    int32_t grid_per_cu; /* persistent workgroups per compute unit, 1..32;    */
                         /* 0: one workgroup per work item (no persistence)  */
} shm_launch_shape;

/* Validates the descriptors (N in range, lut_offset >= 0 and aligned for
 * the dtype/layout, q_begin, q_count >= 0), copies them to the device on
 * `stream` and waits for the copy (objs_host may be released on return),
 * allocates the plan's device memory (the descriptors and a work list sized
 * for the smallest tile a shape may have, 64 queries: sum over objects of
 * ceil(q_count / 64) items of 16 B) and builds the work list with the
 * default shape {256, 2, 2048, 8}.  Apart from the backward's sort buffers
 * (shm_plan_backward_sort) this is the plan's only allocation.
 * The plan must not outlive the device it was created on. */
SHM_API int shm_plan_create(const shm_object* objs_host, int64_t n_obj, int32_t dtype, int32_t layout, hipStream_t stream,
                    shm_plan** plan_out);
/* Times every candidate launch shape on the given (real) buffers, keeps the
 * fastest and returns it in *chosen (may be NULL).  Waits for its own
 * launches on `stream` (and, through shm_plan_set_shape, for the plan's
 * earlier launches).  cache_path: JSON file (host path) that remembers the
 * choice for this workload signature, or NULL. */
SHM_API int shm_plan_autotune(shm_plan* plan, const void* lut, const float* dirs, float* out, const char* cache_path,
                      hipStream_t stream, shm_launch_shape* chosen);
/* Sets the launch shape and drops any captured graph.  It first waits
 * (host) for every launch of the plan's kernel issued so far through
 * shm_plan_launch or shm_plan_graph_launch, on any stream: they may still
 * read the work list or run the graph.  A new tile size then rewrites the
 * work list in place (no allocation).  A graph that the caller captured
 * around shm_plan_launch keeps reading the plan's list: set no new shape
 * while the caller may still replay it. */
SHM_API int shm_plan_set_shape(shm_plan* plan, const shm_launch_shape* shape);
SHM_API int shm_plan_launch(shm_plan* plan, const void* lut, const float* dirs, float* out, float* normal, hipStream_t stream);
/* Captures one shm_plan_launch with these buffers into a HIP graph owned by
 * the plan (replacing an earlier one once the plan's launches so far have
 * completed); shm_plan_graph_launch replays it on `stream`. */
SHM_API int shm_plan_capture_graph(shm_plan* plan, const void* lut, const float* dirs, float* out, float* normal,
                           hipStream_t stream);
SHM_API int shm_plan_graph_launch(shm_plan* plan, hipStream_t stream);
SHM_API int64_t shm_plan_work_items(const shm_plan* plan);
SHM_API int shm_plan_destroy(shm_plan* plan);

/* Backward of a plan's objects (the differentiation form of the batched
 * query; TEXEL plans, FP32 or FP16 LUT): the gradients of Eqs. 4-9 with
 * respect to each object's LUT and to the directions, as shm_query_backward
 * computes them for one object, for objects of their own face sizes, LUT
 * offsets and query ranges.  Each object's LUT gradient has the bits of a
 * one-object shm_query_backward over that object's queries.
 * shm_plan_backward_sort sorts the plan's queries by (object, face, cell)
 * and keeps the sort in the plan; it stays valid while dirs are unchanged.
 * The first call checks that no two objects' LUTs and no two non-empty
 * query ranges overlap (SHM_ERR_INVALID_ARG otherwise), builds the objects'
 * prefix arrays and allocates the sort buffers (44 B per query row up to the
 * last object's range, 4 B per cell and 37 B per gradient tile of 15 x 15
 * texels of all objects); every call first waits
 * (host) for the plan's earlier launches, which may read the sort, and
 * finally for the sort itself (it reads back how many tiles hold a cell of
 * more than 32 queries, which the backward sums by a kernel of their own).
 * shm_plan_backward then, on `stream`:
 *   lut        the objects' LUT (read for the direction gradient only)
 *   grad_out   [rows][4] upstream gradient dL/d(R, g), FP32
 *   grad_lut   dL/dLUT in FP32, the LUT's shape and element offsets (an
 *              FP16 LUT's gradient is FP32 at the same element indices);
 *              every object's texels are overwritten, elements outside all
 *              objects are not touched (or NULL)
 *   grad_dirs  [rows][3] dL/d dirs of every object's rows, NaN for an
 *              invalid direction (or NULL)
 * Deterministic (no floating-point atomics).  Errors: SHM_ERR_UNSUPPORTED
 * for a CELL plan or more than 2^32 - 1 cells or query rows;
 * SHM_ERR_INVALID_ARG for a missing sort, null or misaligned pointers. */
SHM_API int shm_plan_backward_sort(shm_plan* plan, const float* dirs, hipStream_t stream);
SHM_API int shm_plan_backward(shm_plan* plan, const void* lut, const float* dirs, const float* grad_out,
                              float* grad_lut, float* grad_dirs, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Backward (differentiation form) for FP32 TEXEL LUTs with uniform objects
 * as in shm_query_value_grad.  With upstream grad_out[q] = dL/d(R, g):
 *   grad_lut   dL/dLUT, FP32, same shape as lut, overwritten (or NULL)
 *   grad_dirs  dL/d dirs [Q][3] (or NULL); the outputs are 0-homogeneous
 *              in d, so grad_dirs[q] . dirs[q] = 0; NaN for an invalid
 *              direction (zero, NaN or Inf component)
 * grad_lut is deterministic: queries are sorted by cell once (stable: by
 * cell, then by query index); each cell sums its queries' contributions in
 * that order and every texel adds the sums of its <= 4 adjacent cells in a
 * fixed order; no floating-point atomics.  shm_backward_sort builds the sort in the workspace; it stays
 * valid while dirs (and N, n_obj, q_per_obj) are unchanged, so a fitting
 * loop sorts once and passes sort_ready = SHM_SORT_READY afterwards.
 * A tile with a cell of more than 32 queries (dense) is summed by a kernel
 * of its own; the sort lists such tiles.  sort_ready:
 *   0                      sort dirs into the workspace first
 *   SHM_SORT_READY         reuse the sort
 *   SHM_SORT_READY_SPARSE  reuse the sort and launch no dense-tile kernel:
 *                          the tile kernel sums every tile itself.  The
 *                          result is correct either way (equal up to the
 *                          order of the sums), but dense cells are summed
 *                          slowly: pass it when shm_backward_dense_tiles
 *                          returned 0 for this sort.
 * Other values are rejected (SHM_ERR_INVALID_ARG).
 * ---------------------------------------------------------------------- */
#define SHM_SORT_READY 1
#define SHM_SORT_READY_SPARSE 2
SHM_API size_t shm_backward_workspace(int32_t N, int64_t n_obj, int64_t q_per_obj);
/* Cell key of every query: ((obj*6 + face)*(N+1) + j0)*(N+1) + i0, or
 * 0xFFFFFFFF for an invalid direction.  keys [n_obj*q_per_obj] uint32.
 * A caller whose directions stay fixed (a fitting loop) can reorder its
 * queries once by (key, index); the backward's reads of dirs and
 * grad_out are then coalesced. */
SHM_API int shm_cell_keys(int32_t N, int64_t n_obj, const float* dirs, int64_t q_per_obj, uint32_t* keys, hipStream_t stream);
SHM_API int shm_backward_sort(int32_t N, int64_t n_obj, const float* dirs, int64_t q_per_obj, void* ws, size_t ws_bytes,
                      hipStream_t stream);
SHM_API int shm_query_backward(const float* lut, int32_t N, int64_t n_obj, const float* dirs, int64_t q_per_obj,
                       const float* grad_out, float* grad_lut, float* grad_dirs, void* ws, size_t ws_bytes,
                       int32_t sort_ready, hipStream_t stream);
/* The number of dense tiles the sort in ws listed (>= 0), or -1 with an
 * error for bad arguments.  Waits (host) for `stream`, on which the sort was
 * issued: call it once after shm_backward_sort, not per step. */
SHM_API int64_t shm_backward_dense_tiles(int32_t N, int64_t n_obj, int64_t q_per_obj, const void* ws,
                                         size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Ray casting against x(w) = c + R(w) w (Sec. 3.1, Eq. 1), one object.
 * F(t) = |o + t d - c| - R(w), F'(t) = d.w - (d . grad R)/|o + t d - c|.
 * Schedule (fixed counts): bounding sphere |x - c| = rmax -> [t_in, t_out]
 * (miss if none or t_out < 0); march t_k = t0 + k (t_out - t0)/n_march,
 * t0 = max(t_in, 0), k = 1..n_march, the first F(t_k) < 0 brackets the
 * root; n_bisect halvings; n_newton safeguarded Newton steps from the
 * bracket midpoint (a step leaving the closed bracket falls back to its
 * midpoint); one last evaluation at the final t.
 *   center   host float[3];  rmax > 0 must bound R (see shm_lut_rmax)
 *   ray_o, ray_d  [P][3] FP32 (d need not be unit)
 *   t_out    [P] (+inf on a miss);  out [P][4] (R, grad) and normal [P][3]
 *            (may be NULL) at the hit, NaN on a miss
 * n_march + n_bisect + n_newton + 1 <= 64 evaluations per ray.
 * ---------------------------------------------------------------------- */
SHM_API int shm_trace_radial(const void* lut, int32_t dtype, int32_t N, const float* center, float rmax, const float* ray_o,
                     const float* ray_d, int64_t P, int32_t n_march, int32_t n_bisect, int32_t n_newton, float* t_out,
                     float* out, float* normal, hipStream_t stream);

/* The full form (Sec. 3.1): the surface is x(w) = c + R(w) w with the
 * rendered radius R = scale r (scale |r| with SHM_SIGNED, as in
 * shm_query_scaled), and the number of bisections can follow the glyph's
 * projected size.  With px_per_unit > 0 (focal length in pixels), ray k
 * bisects k_b = the fewest halvings that bring e = 2 rmax px_per_unit /
 * (|o_k - c| n_march) pixels (the march bracket's width at the glyph's
 * depth) down to eps_px, at most n_bisect; the decision is FP32 in this
 * order, rounded to nearest without contraction.  px_per_unit = 0 keeps
 * n_bisect fixed.  rmax must bound R (scale * shm_lut_rmax).
 *   sign   [P] int8: sign of r at the hit (0 on a miss) or NULL
 *   evals  [P] uint8: evaluations of F spent by the ray or NULL
 * shm_trace_radial is this with scale 1, no flags, fixed counts and rays
 * in any order. */
typedef struct shm_trace_params {
    float scale;          /* s > 0 */
    int32_t flags;        /* SHM_SIGNED, SHM_CELL_LUT or both, or 0 */
    int32_t n_march;      /* >= 1 */
    int32_t n_bisect;     /* fixed count, or the cap of the adaptive budget */
    int32_t n_newton;     /* n_march + n_bisect + n_newton + 1 <= 64 */
    float px_per_unit;    /* 0: fixed budget; > 0: adaptive */
    float eps_px;         /* > 0 with an adaptive budget */
    int32_t image_width;  /* 0: rays in any order; W > 0: the rays are a
                             row-major image W pixels wide (P a multiple of
                             W) and each wavefront traces an 8 x 8 pixel tile,
                             so that its rays take similar numbers of steps;
                             the results are the same bits either way */
    int32_t bound_blocks; /* 0: no bound map; B in 1..SHM_MAX_BOUND_BLOCKS:
                             bound_map is shm_lut_bound_map's [6][B][B] map
                             of this LUT (same flags), and march samples
                             provably outside the surface (|p - c| above
                             scale x their block's bound) are not evaluated;
                             t, out, normal and sign are the same bits, evals
                             counts only what was evaluated */
    const float* bound_map;
} shm_trace_params;
SHM_API int shm_trace_radial_ex(const void* lut, int32_t dtype, int32_t N, const float* center, float rmax,
                                const shm_trace_params* params, const float* ray_o, const float* ray_d, int64_t P,
                                float* t_out, float* out, float* normal, int8_t* sign, uint8_t* evals,
                                hipStream_t stream);

/* Upper bound of the reconstructed r over one LUT (TEXEL, or CELL with
 * SHM_CELL_LUT: then from the cells as decoded): the largest Bezier control
 * point of any cell's bicubic patch (convex hull property); with
 * SHM_SIGNED the largest |control point|, which bounds |r|.  Writes one
 * float to rmax_out (device). */
SHM_API int shm_lut_rmax(const void* lut, int32_t dtype, int32_t N, int32_t flags, float* rmax_out, hipStream_t stream);

/* Block bound map of one LUT (TEXEL, or CELL with SHM_CELL_LUT) for the
 * trace's empty-space skipping:
 * face f is cut into blocks x blocks blocks of (u, v) (block bi covers
 * u in [bi/blocks, (bi+1)/blocks]); map_out[f][bj][bi] (device, FP32) is
 * the largest Bezier control point (|control point| with SHM_SIGNED), at
 * least 0, over the cells a direction in that block can fall in, widened
 * by one cell on every side.  It bounds r over the block as shm_lut_rmax
 * bounds it over the sphere. */
SHM_API int shm_lut_bound_map(const void* lut, int32_t dtype, int32_t N, int32_t flags, int32_t blocks, float* map_out,
                              hipStream_t stream);

/* ------------------------------------------------------------------------
 * Mip chain (Sec. 4.7, Table lod): the next level (face size N/2, N even) of
 * one FP32 TEXEL LUT.
 *   mode 0 (consistent): the value field is box-filtered -- every coarse
 *     sample is the mean of the level-N map at the four fine texel-centre
 *     directions the coarse texel covers, evaluated as queries (points
 *     beyond the face read the neighbouring face) -- on the coarse padded
 *     grid plus a margin ring, and the derivative channels are recomputed
 *     from the filtered values by central differences (as shm_bake_fd);
 *   mode 1 (naive): as mode 0, but every interior coarse texel holds the
 *     plain average of the four fine texels' stored channels, as a
 *     box-filtering mip generator would.
 *   lut [6][N+2][N+2][4] -> out [6][N/2+2][N/2+2][4]; ws of
 *   shm_mip_level_workspace(N) bytes (the filtered samples).
 * ---------------------------------------------------------------------- */
SHM_API size_t shm_mip_level_workspace(int32_t N);
SHM_API int shm_mip_level(const float* lut, int32_t N, int32_t mode, void* ws, size_t ws_bytes, float* out,
                          hipStream_t stream);

/* ------------------------------------------------------------------------
 * Radial depth of a triangle mesh (Sec. 4.9, mesh LOD impostors):
 * depth[k] = max{t >= 0 : c + t w_k on the mesh surface}, w_k = dirs[k]
 * normalised, 0 when the ray from c meets no triangle (or w_k is zero,
 * NaN or Inf).  Every triangle is tested (a ray cast against the whole
 * mesh, FP32; a hit needs barycentrics >= -4 ulp, so rays through shared
 * edges are not lost).  Triangles with an index outside [0, n_verts) are
 * skipped.  With the directions of shm_margin_dirs(N) and shm_bake_fd this
 * bakes the mesh's impostor LUT.
 *   verts  [n_verts][3] FP32;  tris [n_tris][3] int32;  center host float[3]
 *   dirs   [P][3] FP32;  depth [P] FP32 (written)
 * ---------------------------------------------------------------------- */
SHM_API int shm_mesh_radial_depth(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                                  const float* center, const float* dirs, int64_t P, float* depth,
                                  hipStream_t stream);

/* ------------------------------------------------------------------------
 * Comparison paths of the paper's experiments (Sec. 4.2, 4.5, 4.6; Tables
 * psnr_value, cost_extended, runtime), on the same GPU as the Hermite query.
 * shm_query_baseline reconstructs from a value-only LUT
 *   vlut [n_obj][6][N+4][N+4] FP32, texel p at u = (p - 3/2)/N (a two-texel
 *   gutter; exactly the samples at shm_margin_dirs(N)):
 *   SHM_RECON_NEAREST      nearest texel, zero gradient (1 fetch)
 *   SHM_RECON_BILINEAR_FD  bilinear value, chart derivatives by central
 *                          differences of 4 more bilinear lookups at u +- h,
 *                          v +- h
 *   SHM_RECON_BICUBIC      16-tap Catmull-Rom value and analytic gradient
 *   SHM_RECON_FAST_BICUBIC_FD  "fast bicubic" (Table cost_extended): the
 *                          cubic B-spline of the samples (what 4 hardware
 *                          bilinear fetches evaluate; FP32 weights here),
 *                          gradient as in SHM_RECON_BILINEAR_FD
 * Without texture units, all but nearest read the cell's 4 x 4 footprint
 * once (the +-1 texel bilinear lookups fall inside it): 16 scalars.
 * then transports (r_u, r_v) to the spherical gradient as the Hermite query
 * does.  shm_sh_eval evaluates sum_k coeffs[k] Y_k and its spherical
 * gradient directly, without a LUT (coeffs [n_obj][(L+1)^2], L <= 16).
 * Both write out [n_obj*q_per_obj][4] = (R, gx, gy, gz); NaN for invalid
 * directions.
 * ---------------------------------------------------------------------- */
typedef enum {
    SHM_RECON_NEAREST = 0,
    SHM_RECON_BILINEAR_FD = 1,
    SHM_RECON_BICUBIC = 2,
    SHM_RECON_FAST_BICUBIC_FD = 3
} shm_recon;
SHM_API int shm_query_baseline(const float* vlut, int32_t N, int64_t n_obj, const float* dirs, int64_t q_per_obj,
                               int32_t method, float* out, hipStream_t stream);
SHM_API int shm_sh_eval(const float* coeffs, int32_t L, int64_t n_obj, const float* dirs, int64_t q_per_obj,
                        float* out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Fitting a LUT to a target (the differentiation form): the two steps of
 * the optimisation loop around shm_query_value_grad (TEXEL, FP32) and
 * shm_query_backward, so that a whole step runs in this library's kernels
 * (no allocation, no host synchronisation: a fixed sequence of steps can be
 * captured in a graph; the step number t is a launch argument).
 *
 * shm_fit_loss_grad writes dL/d(R, gx, gy, gz) for the objective
 *   L = w_value mean_q (R_q - target_r[q])^2 + mean_q |n_q - target_n[q]|^2
 * with n = (R w - grad R) / |R w - grad R| (Eq. 10), w = d/|d|:
 *   out      [Q][4] the query's output (R, grad R), 16-byte aligned
 *   dirs     [Q][3] the query directions
 *   target_r [Q], target_n [Q][3] (unit normals)
 *   grad     [Q][4] written (16-byte aligned); 0 for queries whose output
 *            is not finite (zero or non-finite directions) or whose
 *            R w - grad R vanishes
 * shm_adam_step applies one Adam update in place to a FP32 TEXEL LUT
 * param [n4][4] (n4 texels; channel 0 = r uses lr_value, channels 1..3 =
 * the scaled derivatives use lr_deriv), with gradient grad and moment
 * buffers m, v of the same shape (zero before step 1), step t >= 1:
 *   m <- m + (1 - beta1)(g - m),  v <- beta2 v + (1 - beta2) g^2,
 *   p <- p - lr / (1 - beta1^t) * m / (sqrt(v) / sqrt(1 - beta2^t) + eps).
 * All four arrays 16-byte aligned; 0 <= beta1, beta2 < 1, eps > 0.
 * ---------------------------------------------------------------------- */
SHM_API int shm_fit_loss_grad(const float* out, const float* dirs, const float* target_r, const float* target_n,
                              int64_t Q, float w_value, float* grad, hipStream_t stream);
/* The forward query of one FP32 TEXEL LUT (face size N) fused with
 * shm_fit_loss_grad: grad as above for out = the query of lut at dirs,
 * without writing out (lut 16-byte aligned). */
SHM_API int shm_fit_forward_loss_grad(const float* lut, int32_t N, const float* dirs, const float* target_r,
                                      const float* target_n, int64_t Q, float w_value, float* grad,
                                      hipStream_t stream);
SHM_API int shm_adam_step(float* param, const float* grad, float* m, float* v, int64_t n4, int64_t step,
                          float lr_value, float lr_deriv, float beta1, float beta2, float eps, hipStream_t stream);
/* One whole fitting step of one FP32 TEXEL LUT (face size N) in one kernel:
 * the forward query of lut_in at dirs, the objective's gradient as in
 * shm_fit_loss_grad, the LUT gradient as in shm_query_backward (the same
 * sorted, deterministic sums; no direction gradient) and the Adam update as
 * in shm_adam_step, written to lut_out:
 *   lut_out = adam(lut_in, dL/dLUT(lut_in), m, v, step)
 *   lut_in, lut_out  [6][N+2][N+2][4]; lut_out is overwritten and must not
 *            overlap lut_in (a texel's update and its neighbours' queries
 *            run concurrently), so a loop alternates two buffers
 *   m, v     Adam moments of the same shape, updated in place (zero before
 *            step 1); none of the four buffers may overlap another
 *   dirs, target_r, target_n, Q, w_value  as in shm_fit_loss_grad
 *   step, lr_value, lr_deriv, beta1, beta2, eps  as in shm_adam_step
 *   ws, ws_bytes  shm_backward_workspace(N, 1, Q) bytes, 256-byte aligned;
 *            sort_ready = 0 sorts dirs into it first, SHM_SORT_READY reuses
 *            the sort a previous call (or shm_backward_sort(N, 1, dirs, Q))
 *            left there, SHM_SORT_READY_SPARSE as for shm_query_backward
 * Q = 0 is allowed: the gradient is zero and Adam still moves the moments. */
SHM_API int shm_fit_step(const float* lut_in, float* lut_out, float* m, float* v, int32_t N, const float* dirs,
                         const float* target_r, const float* target_n, int64_t Q, float w_value, int64_t step,
                         float lr_value, float lr_deriv, float beta1, float beta2, float eps, void* ws,
                         size_t ws_bytes, int32_t sort_ready, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SHM_H */
