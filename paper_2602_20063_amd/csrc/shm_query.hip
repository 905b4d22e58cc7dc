// Query kernels: value + spherical gradient from a Spherical Hermite Map
// (Sec. 3.2-3.4).  One lane answers one query: locate -> 16-scalar gather ->
// Hermite patch -> closed-form metric transport -> coalesced float4 store.
//
// The query is bound by HBM traffic: every query's footprint is one random
// gather of 64 B (FP32) or 32 B (FP16), and HBM serves random requests in
// 128 B lines, so the CELL layout (footprint contiguous and aligned, one
// line per query) is what the throughput path uses; the TEXEL layout is
// served by the same kernel (two 32 B row segments per query).
#include "shm_device.hpp"
#include "shm_internal.hpp"

// Compile-time tuning knobs of the uniform kernel (every setting gives the
// same bits; the measured sweep is recorded with the design notes):
//   SHM_QPT     queries per lane (2 or more: the batched form, query_batch)
//   SHM_QBLOCK  lanes per workgroup (one tile = SHM_QBLOCK * SHM_QPT queries)
//   SHM_DIR_NT  non-temporal direction loads
//   SHM_OUT_NT  non-temporal result stores
// Both streams are touched once; non-temporal accesses keep them from
// displacing the LUT lines in L2/MALL (non-temporal LUT loads are slower).
#ifndef SHM_QPT
#define SHM_QPT 1
#endif
#ifndef SHM_QBLOCK
#define SHM_QBLOCK 256
#endif
#ifndef SHM_DIR_NT
#define SHM_DIR_NT 1
#endif
#ifndef SHM_OUT_NT
#define SHM_OUT_NT 1
#endif

namespace shm {

constexpr int QB = SHM_QBLOCK;

__device__ __forceinline__ float ld_dir(const float* p)
{
#if SHM_DIR_NT
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

__device__ __forceinline__ void st_out(float* out, int64_t q, float4 r)
{
#if SHM_OUT_NT
    __builtin_nontemporal_store(f32x4{r.x, r.y, r.z, r.w}, reinterpret_cast<f32x4*>(out) + q);
#else
    reinterpret_cast<float4*>(out)[q] = r;
#endif
}


// QPT queries per lane: rows q0 + k0 + j B + lane (j < QPT) of a range of
// n rows.  All their loads go out before any query's arithmetic, with no
// branch between them (a branch ends in a wait for every load in flight),
// so a lane has QPT footprints in flight; an idle lane (row >= n) reads the
// range's first direction.  Results (and normals) are written through
// buffer descriptors ro (rn) whose ranges end at the range's last row: the
// stores of idle lanes fall outside them and are dropped, so no branch
// guards a store (aux 2: non-temporal).  The same bits as query_one.
template <bool FP16, bool CELL, bool NRM, int QPT>
__device__ __forceinline__ void query_batch(const char* __restrict__ base, int N, const float* __restrict__ dirs,
                                            int64_t q0, int n, int k0, int B, __amdgpu_buffer_rsrc_t ro,
                                            __amdgpu_buffer_rsrc_t rn)
{
    float x[QPT], y[QPT], z[QPT];
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        const int k = k0 + j * B + (int)threadIdx.x;
        const int64_t q = q0 + (k < n ? k : 0);
        x[j] = ld_dir(dirs + 3 * q);
        y[j] = ld_dir(dirs + 3 * q + 1);
        z[j] = ld_dir(dirs + 3 * q + 2);
    }
    // an empty statement that takes (and may change) every loaded value: no
    // query's arithmetic can start before all the loads above are issued
#pragma unroll
    for (int j = 0; j < QPT; ++j) asm volatile("" : "+v"(x[j]), "+v"(y[j]), "+v"(z[j]));
    Loc L[QPT];
    Foot F[QPT];
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        L[j] = locate(x[j], y[j], z[j], N);
        F[j] = decode<FP16, CELL>(query_load<FP16, CELL>(base, N, L[j]));
    }
#pragma unroll
    for (int j = 0; j < QPT; ++j) pin(F[j]);
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        const uint32_t k = (uint32_t)(k0 + j * B + (int)threadIdx.x);
        const float4 r = query_finish(F[j], L[j], N);
        const u32x4 w = {__float_as_uint(r.x), __float_as_uint(r.y), __float_as_uint(r.z), __float_as_uint(r.w)};
        __builtin_amdgcn_raw_buffer_store_b128(w, ro, k * 16u, 0, 2);
        if constexpr (NRM) {
            const float3 nv = normal_of(r.x, x[j], y[j], z[j], make_float3(r.y, r.z, r.w));
            const u32x3 wn = {__float_as_uint(nv.x), __float_as_uint(nv.y), __float_as_uint(nv.z)};
            __builtin_amdgcn_raw_buffer_store_b96(wn, rn, k * 12u, 0, 2);
        }
    }
}

template <bool FP16, bool CELL, bool NRM>
__global__ __launch_bounds__(QB) void k_query_uniform(const void* __restrict__ lut, int N, int64_t lut_elems,
                                                       int64_t q_per_obj, int tiles_per_obj,
                                                       const float* __restrict__ dirs, float* __restrict__ out,
                                                       float* __restrict__ nrm)
{
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int obj = b / tiles_per_obj;
    const int tile = b - obj * tiles_per_obj;
    const char* base = reinterpret_cast<const char*>(lut) + (size_t)obj * (size_t)lut_elems * (FP16 ? 2 : 4);
    if constexpr (SHM_QPT > 1) {
        const int64_t ql0 = (int64_t)tile * (QB * SHM_QPT);
        const int64_t q0 = (int64_t)obj * q_per_obj + ql0;
        const int n = (int)((q_per_obj - ql0) < QB * SHM_QPT ? (q_per_obj - ql0) : QB * SHM_QPT);
        const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(out + 4 * q0, (short)0, n * 16, 0x00020000);
        const __amdgpu_buffer_rsrc_t rn =
            __builtin_amdgcn_make_buffer_rsrc(NRM ? nrm + 3 * q0 : out, (short)0, NRM ? n * 12 : 0, 0x00020000);
        query_batch<FP16, CELL, NRM, SHM_QPT>(base, N, dirs, q0, n, 0, QB, ro, rn);
        return;
    }
    float x[SHM_QPT], y[SHM_QPT], z[SHM_QPT];
    int64_t qq[SHM_QPT];
    bool act[SHM_QPT];
#pragma unroll
    for (int j = 0; j < SHM_QPT; ++j) {
        const int64_t ql = (int64_t)tile * (QB * SHM_QPT) + j * QB + threadIdx.x;
        act[j] = ql < q_per_obj;
        qq[j] = (int64_t)obj * q_per_obj + ql;
        if (act[j]) {
            x[j] = ld_dir(dirs + 3 * qq[j]);
            y[j] = ld_dir(dirs + 3 * qq[j] + 1);
            z[j] = ld_dir(dirs + 3 * qq[j] + 2);
        }
    }
#pragma unroll
    for (int j = 0; j < SHM_QPT; ++j) {
        if (!act[j]) continue;
        const float4 r = query_one<FP16, CELL>(base, N, x[j], y[j], z[j]);
        st_out(out, qq[j], r);
        if constexpr (NRM) {
            const float3 n = normal_of(r.x, x[j], y[j], z[j], make_float3(r.y, r.z, r.w));
            nrm[3 * qq[j]] = n.x;
            nrm[3 * qq[j] + 1] = n.y;
            nrm[3 * qq[j] + 2] = n.z;
        }
    }
}

// Step a3 alone (Sec. 3.2): the 16 footprint scalars of every query, with
// the launch mapping, the cell decision and the loads of k_query_uniform,
// written as 4 float4 (corners (i0,j0), (i0+1,j0), (i0,j0+1), (i0+1,j0+1),
// each (r, r_u h, r_v h, r_uv h^2)); NaN for an invalid direction.
template <bool FP16, bool CELL>
__global__ __launch_bounds__(QB) void k_gather_foot(const void* __restrict__ lut, int N, int64_t lut_elems,
                                                     int64_t q_per_obj, int tiles_per_obj,
                                                     const float* __restrict__ dirs, float4* __restrict__ foot)
{
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int obj = b / tiles_per_obj;
    const int tile = b - obj * tiles_per_obj;
    const char* base = reinterpret_cast<const char*>(lut) + (size_t)obj * (size_t)lut_elems * (FP16 ? 2 : 4);
    float x[SHM_QPT], y[SHM_QPT], z[SHM_QPT];
    int64_t qq[SHM_QPT];
    bool act[SHM_QPT];
#pragma unroll
    for (int j = 0; j < SHM_QPT; ++j) {
        const int64_t ql = (int64_t)tile * (QB * SHM_QPT) + j * QB + threadIdx.x;
        act[j] = ql < q_per_obj;
        qq[j] = (int64_t)obj * q_per_obj + ql;
        if (act[j]) {
            x[j] = ld_dir(dirs + 3 * qq[j]);
            y[j] = ld_dir(dirs + 3 * qq[j] + 1);
            z[j] = ld_dir(dirs + 3 * qq[j] + 2);
        }
    }
#pragma unroll
    for (int j = 0; j < SHM_QPT; ++j) {
        if (!act[j]) continue;
        const Loc L = locate(x[j], y[j], z[j], N);
        Foot F;
        if (L.face < 0) {
            const float nan = __builtin_nanf("");
#pragma unroll
            for (int k = 0; k < 4; ++k) F.c[k] = make_float4(nan, nan, nan, nan);
        } else {
            F = load_foot<FP16, CELL>(base, N, L);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) foot[4 * qq[j] + k] = F.c[k];
    }
}

int launch_gather_footprints(const void* lut, int dtype, int layout, int N, int64_t n_obj, const float* dirs,
                             int64_t q_per_obj, float* foot, hipStream_t stream)
{
    if (n_obj == 0 || q_per_obj == 0) return SHM_OK;
    const int64_t tiles = (q_per_obj + QB * SHM_QPT - 1) / (QB * SHM_QPT);
    if (tiles > 0x7fffffff || tiles * n_obj > 0x7fffffff)
        return fail(SHM_ERR_UNSUPPORTED, "gather_footprints: %lld objects x %lld tiles exceeds one launch",
                    (long long)n_obj, (long long)tiles);
    const dim3 grid((unsigned)(tiles * n_obj));
    const int64_t le = layout == SHM_LAYOUT_CELL ? cell_elems(N) : texel_elems(N);
    float4* f4 = reinterpret_cast<float4*>(foot);
    const int tpo = (int)tiles;
    if (dtype == SHM_F16) {
        if (layout == SHM_LAYOUT_CELL) hipLaunchKernelGGL((k_gather_foot<true, true>), grid, dim3(QB), 0, stream, lut, N, le, q_per_obj, tpo, dirs, f4);
        else hipLaunchKernelGGL((k_gather_foot<true, false>), grid, dim3(QB), 0, stream, lut, N, le, q_per_obj, tpo, dirs, f4);
    } else {
        if (layout == SHM_LAYOUT_CELL) hipLaunchKernelGGL((k_gather_foot<false, true>), grid, dim3(QB), 0, stream, lut, N, le, q_per_obj, tpo, dirs, f4);
        else hipLaunchKernelGGL((k_gather_foot<false, false>), grid, dim3(QB), 0, stream, lut, N, le, q_per_obj, tpo, dirs, f4);
    }
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

template <bool FP16, bool CELL, bool NRM>
static void launch_uniform_t(dim3 grid, hipStream_t st, const void* lut, int N, int64_t le, int64_t qpo, int tpo,
                             const float* dirs, float* out, float* nrm)
{
    hipLaunchKernelGGL((k_query_uniform<FP16, CELL, NRM>), grid, dim3(QB), 0, st, lut, N, le, qpo, tpo, dirs, out,
                       nrm);
}

int launch_query_uniform(const void* lut, int dtype, int layout, int N, int64_t n_obj, const float* dirs,
                         int64_t q_per_obj, float* out, float* normal, hipStream_t stream)
{
    if (n_obj == 0 || q_per_obj == 0) return SHM_OK;
    const int64_t tiles = (q_per_obj + QB * SHM_QPT - 1) / (QB * SHM_QPT);
    if (tiles > 0x7fffffff || tiles * n_obj > 0x7fffffff)
        return fail(SHM_ERR_UNSUPPORTED, "query: %lld objects x %lld tiles exceeds one launch", (long long)n_obj,
                    (long long)tiles);
    const dim3 grid((unsigned)(tiles * n_obj));
    const int64_t le = layout == SHM_LAYOUT_CELL ? cell_elems(N) : texel_elems(N);
    const bool f16 = dtype == SHM_F16, cell = layout == SHM_LAYOUT_CELL, nrm = normal != nullptr;
    const int tpo = (int)tiles;
#define SHM_Q(a, b, c) launch_uniform_t<a, b, c>(grid, stream, lut, N, le, q_per_obj, tpo, dirs, out, normal)
    if (f16) {
        if (cell) { if (nrm) SHM_Q(true, true, true); else SHM_Q(true, true, false); }
        else { if (nrm) SHM_Q(true, false, true); else SHM_Q(true, false, false); }
    } else {
        if (cell) { if (nrm) SHM_Q(false, true, true); else SHM_Q(false, true, false); }
        else { if (nrm) SHM_Q(false, false, true); else SHM_Q(false, false, false); }
    }
#undef SHM_Q
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

// ---------------------------------------------------------------------------
// Persistent batched kernel.  The work list holds (object, query range)
// items of at most `tile` queries, ordered by object, and is cut into 8
// contiguous slices of equal query counts; the workgroups of one XCD take
// the items of one slice in turn (static striding: deterministic, no
// counters, nothing to reset, so a captured graph replays as is).  Items
// processed at the same time are neighbours in the list, so an object's LUT
// is read by the workgroups of one XCD and stays resident in its L2.
// ---------------------------------------------------------------------------
template <bool FP16, bool CELL, bool NRM, int QPT>
__global__ void k_query_persistent(const void* __restrict__ lut, const shm_object* __restrict__ objs,
                                   const WorkItem* __restrict__ items, XcdSplit split,
                                   const float* __restrict__ dirs, float* __restrict__ out, float* __restrict__ nrm)
{
    // nx groups of blocks (the XCDs, or all G blocks when G < 8); group x
    // has per blocks and walks slices x, x + nx, ... of the work list
    const int G = (int)gridDim.x;
    const int nx = G < 8 ? G : 8;
    const int x = (int)blockIdx.x % nx, local = (int)blockIdx.x / nx;
    const int per = (G - x + nx - 1) / nx;
    const int B = (int)blockDim.x;
    for (int s = x; s < 8; s += nx)
    for (int64_t w = split.b[s] + local; w < split.b[s + 1]; w += per) {
        const WorkItem it = items[w];
        const shm_object o = objs[it.obj];
        const int N = o.N;
        const char* base = reinterpret_cast<const char*>(lut) + (size_t)o.lut_offset * (FP16 ? 2 : 4);
        if constexpr (QPT == 1) {
            // one query per lane: each lane's loads are serial anyway (the
            // direction decides the cell), and the plain form measures fastest
            for (int k0 = 0; k0 < it.n; k0 += B) {
                const int k = k0 + (int)threadIdx.x;
                if (k >= it.n) continue;
                const int64_t q = it.q0 + k;
                const float x = ld_dir(dirs + 3 * q), y = ld_dir(dirs + 3 * q + 1), z = ld_dir(dirs + 3 * q + 2);
                const float4 r = query_one<FP16, CELL>(base, N, x, y, z);
                st_out(out, q, r);
                if constexpr (NRM) {
                    const float3 n = normal_of(r.x, x, y, z, make_float3(r.y, r.z, r.w));
                    nrm[3 * q] = n.x;
                    nrm[3 * q + 1] = n.y;
                    nrm[3 * q + 2] = n.z;
                }
            }
            continue;
        }
        // QPT queries per lane, all loads before any arithmetic (query_batch)
        const __amdgpu_buffer_rsrc_t ro =
            __builtin_amdgcn_make_buffer_rsrc(out + 4 * it.q0, (short)0, it.n * 16, 0x00020000);
        const __amdgpu_buffer_rsrc_t rn =
            __builtin_amdgcn_make_buffer_rsrc(NRM ? nrm + 3 * it.q0 : out, (short)0, NRM ? it.n * 12 : 0, 0x00020000);
        for (int k0 = 0; k0 < it.n; k0 += B * QPT)
            query_batch<FP16, CELL, NRM, QPT>(base, N, dirs, it.q0, it.n, k0, B, ro, rn);
    }
}

// ---------------------------------------------------------------------------
// Plan-free query of objects described on the device.  k_obj_tiles counts
// each object's tiles of OBJ_TILE queries (0 for an object the kernel would
// skip) and scans the counts in one workgroup into tile_start[0..n_obj];
// k_query_objects then walks tiles 0 .. tile_start[n_obj) - 1 with a
// persistent grid, the tiles cut into 8 contiguous slices, one per XCD
// (group of blocks blockIdx % 8), so an object's tiles share one L2.  A
// workgroup finds the object of its tile by binary search over tile_start
// (uniform across the workgroup).  Deterministic: every query is answered
// by query_one exactly as the uniform and plan kernels answer it.
// ---------------------------------------------------------------------------
// launch shape of the plan-free kernel (compile-time knobs, same bits at any
// setting): queries per lane, workgroups per compute unit
#ifndef SHM_OBJ_QPT
#define SHM_OBJ_QPT 4
#endif
#ifndef SHM_OBJ_WG_PER_CU
#define SHM_OBJ_WG_PER_CU 4
#endif
constexpr int OBJ_LANES = 256;
constexpr int OBJ_TILE = OBJ_LANES * SHM_OBJ_QPT;  // queries per tile
constexpr int OBJ_SCAN = 1024;                     // lanes of the scan workgroup

// an object the kernel answers: N in range, the LUT offset aligned for the
// loads of the dtype/layout, a nonnegative range
template <bool FP16, bool CELL>
__device__ __forceinline__ bool obj_ok(const shm_object& o)
{
    const int64_t al = (FP16 && CELL) ? 8 : 4;
    return o.N >= 1 && o.N <= SHM_MAX_N && o.lut_offset >= 0 && o.lut_offset % al == 0 && o.q_begin >= 0 &&
           o.q_count > 0;
}

template <bool FP16, bool CELL>
__global__ __launch_bounds__(OBJ_SCAN) void k_obj_tiles(const shm_object* __restrict__ objs, int64_t n_obj,
                                                        int64_t* __restrict__ tile_start)
{
    __shared__ int64_t part[OBJ_SCAN];
    const int tid = threadIdx.x;
    const int64_t per = (n_obj + OBJ_SCAN - 1) / OBJ_SCAN;
    const int64_t b = tid * per, e = min(b + per, n_obj);
    int64_t sum = 0;
    for (int64_t o = b; o < e; ++o) {
        const shm_object ob = objs[o];
        sum += obj_ok<FP16, CELL>(ob) ? (ob.q_count + OBJ_TILE - 1) / OBJ_TILE : 0;
    }
    part[tid] = sum;
    __syncthreads();
    // inclusive scan of the lane sums (Hillis-Steele; exact integers)
    for (int d = 1; d < OBJ_SCAN; d <<= 1) {
        const int64_t v = tid >= d ? part[tid - d] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = tid > 0 ? part[tid - 1] : 0;
    for (int64_t o = b; o < e; ++o) {
        tile_start[o] = run;
        const shm_object ob = objs[o];
        run += obj_ok<FP16, CELL>(ob) ? (ob.q_count + OBJ_TILE - 1) / OBJ_TILE : 0;
    }
    if (tid == OBJ_SCAN - 1) tile_start[n_obj] = part[OBJ_SCAN - 1];
}

template <bool FP16, bool CELL, bool NRM>
__global__ __launch_bounds__(OBJ_LANES) void k_query_objects(const void* __restrict__ lut,
                                                            const shm_object* __restrict__ objs, int64_t n_obj,
                                                            const int64_t* __restrict__ tile_start,
                                                            const float* __restrict__ dirs, float* __restrict__ out,
                                                            float* __restrict__ nrm)
{
    const int64_t total = tile_start[n_obj];
    const int G = (int)gridDim.x;
    const int nx = G < 8 ? G : 8;
    const int x = (int)blockIdx.x % nx, local = (int)blockIdx.x / nx;
    const int per = (G - x + nx - 1) / nx;
    // slice x of the tiles: [total x / nx, total (x + 1) / nx)
    const int64_t t_end = total * (x + 1) / nx;
    for (int64_t t = total * x / nx + local; t < t_end; t += per) {
        // the object of tile t: the last o with tile_start[o] <= t (objects
        // without tiles share their successor's start)
        int64_t lo = 0, hi = n_obj - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (tile_start[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const shm_object o = objs[lo];
        const char* base = reinterpret_cast<const char*>(lut) + (size_t)o.lut_offset * (FP16 ? 2 : 4);
        const int64_t k0 = (t - tile_start[lo]) * OBJ_TILE + threadIdx.x;
        float x0[SHM_OBJ_QPT], y0[SHM_OBJ_QPT], z0[SHM_OBJ_QPT];
#pragma unroll
        for (int j = 0; j < SHM_OBJ_QPT; ++j) {
            const int64_t k = k0 + j * OBJ_LANES;
            if (k < o.q_count) {
                const int64_t q = o.q_begin + k;
                x0[j] = ld_dir(dirs + 3 * q);
                y0[j] = ld_dir(dirs + 3 * q + 1);
                z0[j] = ld_dir(dirs + 3 * q + 2);
            }
        }
#pragma unroll
        for (int j = 0; j < SHM_OBJ_QPT; ++j) {
            const int64_t k = k0 + j * OBJ_LANES;
            if (k >= o.q_count) continue;
            const int64_t q = o.q_begin + k;
            const float4 r = query_one<FP16, CELL>(base, o.N, x0[j], y0[j], z0[j]);
            st_out(out, q, r);
            if constexpr (NRM) {
                const float3 n = normal_of(r.x, x0[j], y0[j], z0[j], make_float3(r.y, r.z, r.w));
                nrm[3 * q] = n.x;
                nrm[3 * q + 1] = n.y;
                nrm[3 * q + 2] = n.z;
            }
        }
    }
}

template <bool FP16, bool CELL, bool NRM>
static void launch_objects_t(int n_cu, hipStream_t st, const void* lut, const shm_object* objs, int64_t n_obj,
                             int64_t* tile_start, const float* dirs, float* out, float* nrm)
{
    hipLaunchKernelGGL((k_obj_tiles<FP16, CELL>), dim3(1), dim3(OBJ_SCAN), 0, st, objs, n_obj, tile_start);
    hipLaunchKernelGGL((k_query_objects<FP16, CELL, NRM>), dim3((unsigned)(n_cu * SHM_OBJ_WG_PER_CU)), dim3(OBJ_LANES), 0,
                       st, lut, objs, n_obj, tile_start, dirs, out, nrm);
}

size_t query_objects_workspace(int64_t n_obj) { return (size_t)(n_obj + 1) * sizeof(int64_t); }

int launch_query_objects(const void* lut, int dtype, int layout, const shm_object* objs, int64_t n_obj,
                         const float* dirs, float* out, float* normal, void* ws, hipStream_t stream)
{
    if (n_obj == 0) return SHM_OK;
    int64_t* ts = reinterpret_cast<int64_t*>(ws);
    const int n_cu = device_cu_count();
    const bool f16 = dtype == SHM_F16, cell = layout == SHM_LAYOUT_CELL, nrm = normal != nullptr;
#define SHM_O(a, b, c) launch_objects_t<a, b, c>(n_cu, stream, lut, objs, n_obj, ts, dirs, out, normal)
    if (f16) {
        if (cell) { if (nrm) SHM_O(true, true, true); else SHM_O(true, true, false); }
        else { if (nrm) SHM_O(true, false, true); else SHM_O(true, false, false); }
    } else {
        if (cell) { if (nrm) SHM_O(false, true, true); else SHM_O(false, true, false); }
        else { if (nrm) SHM_O(false, false, true); else SHM_O(false, false, false); }
    }
#undef SHM_O
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

template <bool FP16, bool CELL, bool NRM>
static void launch_persistent_t(int qpt, dim3 grid, dim3 block, hipStream_t st, const void* lut,
                                const shm_object* objs, const WorkItem* items, const XcdSplit& split, const float* dirs,
                                float* out, float* nrm)
{
    switch (qpt) {
    case 1: hipLaunchKernelGGL((k_query_persistent<FP16, CELL, NRM, 1>), grid, block, 0, st, lut, objs, items, split, dirs, out, nrm); break;
    case 2: hipLaunchKernelGGL((k_query_persistent<FP16, CELL, NRM, 2>), grid, block, 0, st, lut, objs, items, split, dirs, out, nrm); break;
    default: hipLaunchKernelGGL((k_query_persistent<FP16, CELL, NRM, 4>), grid, block, 0, st, lut, objs, items, split, dirs, out, nrm); break;
    }
}

int launch_query_persistent(const void* lut, int dtype, int layout, const shm_object* objs_dev,
                            const WorkItem* items_dev, int64_t n_items, const XcdSplit& split,
                            const shm_launch_shape& shape, int n_cu, const float* dirs, float* out, float* normal,
                            hipStream_t stream)
{
    if (n_items == 0) return SHM_OK;
    // grid_per_cu 0: one workgroup per work item (each runs its item and
    // exits: no store of one item waits behind the loads of the next)
    const int64_t G = plan_grid(shape, n_cu, n_items, split);
    const dim3 grid((unsigned)G), block((unsigned)shape.block);
    const bool f16 = dtype == SHM_F16, cell = layout == SHM_LAYOUT_CELL, nrm = normal != nullptr;
#define SHM_P(a, b, c) launch_persistent_t<a, b, c>(shape.qpt, grid, block, stream, lut, objs_dev, items_dev, split, dirs, out, normal)
    if (f16) {
        if (cell) { if (nrm) SHM_P(true, true, true); else SHM_P(true, true, false); }
        else { if (nrm) SHM_P(true, false, true); else SHM_P(true, false, false); }
    } else {
        if (cell) { if (nrm) SHM_P(false, true, true); else SHM_P(false, true, false); }
        else { if (nrm) SHM_P(false, false, true); else SHM_P(false, false, false); }
    }
#undef SHM_P
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

// ---------------------------------------------------------------------------
// TEXEL -> CELL relayout: one lane per (cell, corner), 16 B (FP32) or 8 B
// (FP16) written contiguously.  FP16 cells hold the value channel of corners
// 1..3 as differences from corner 0's value (FP16 cell encoding, see
// decode()); from FP16 texels the difference is formed in FP32 (exact)
// and rounded once.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint2 f4_to_h4(float4 v)
{
    const __half2 lo = __floats2half2_rn(v.x, v.y), hi = __floats2half2_rn(v.z, v.w);
    return make_uint2(*reinterpret_cast<const uint32_t*>(&lo), *reinterpret_cast<const uint32_t*>(&hi));
}

template <typename V>
__global__ void k_lut_to_cells(const V* __restrict__ tex, int N, int64_t total, V* __restrict__ cells)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int corner = (int)(i & 3);
    const int64_t cell = i >> 2;
    const int C = N + 1, P = N + 2;
    const int64_t per_obj = 6ll * C * C;
    const int64_t obj = cell / per_obj;
    int64_t r = cell - obj * per_obj;
    const int face = (int)(r / ((int64_t)C * C));
    r -= (int64_t)face * C * C;
    const int j0 = (int)(r / C), i0 = (int)(r - (int64_t)j0 * C);
    const int p = i0 + (corner & 1), q = j0 + (corner >> 1);
    const int64_t t0 = obj * (6ll * P * P) + ((int64_t)face * P + j0) * P + i0;
    const V v = tex[obj * (6ll * P * P) + ((int64_t)face * P + q) * P + p];
    if constexpr (sizeof(V) == 8) {  // FP16: value of corners 1..3 as a difference
        if (corner > 0) {
            float4 f = h4_to_f4(v);
            f.x -= h4_to_f4(tex[t0]).x;
            cells[i] = f4_to_h4(f);
            return;
        }
    }
    cells[i] = v;
}

// FP32 cells (any run of whole cells, mixed face sizes included) -> FP16
// cells: the value of corners 1..3 as its difference from corner 0's value,
// formed in FP32 and rounded once; every other channel rounded once.
__global__ void k_cells_to_f16(const float4* __restrict__ src, int64_t n_cells, uint2* __restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_cells * 4) return;
    float4 v = src[i];
    if ((i & 3) != 0) v.x -= src[i & ~(int64_t)3].x;
    dst[i] = f4_to_h4(v);
}

int launch_cells_to_f16(const float* cells, int64_t n_cells, void* cells_f16, hipStream_t stream)
{
    if (n_cells == 0) return SHM_OK;
    const int64_t blocks = (n_cells * 4 + 255) / 256;
    if (blocks > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "cells_to_f16: too large");
    hipLaunchKernelGGL(k_cells_to_f16, dim3((unsigned)blocks), dim3(256), 0, stream,
                       reinterpret_cast<const float4*>(cells), n_cells, reinterpret_cast<uint2*>(cells_f16));
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

int launch_lut_to_cells(const void* lut, int dtype, int N, int64_t n_obj, void* cells, hipStream_t stream)
{
    const int64_t total = n_obj * 6ll * (N + 1) * (N + 1) * 4;  // (cell, corner) pairs
    if (total == 0) return SHM_OK;
    const int64_t blocks = (total + 255) / 256;
    if (blocks > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "lut_to_cells: too large");
    if (dtype == SHM_F16)
        hipLaunchKernelGGL(k_lut_to_cells<uint2>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           reinterpret_cast<const uint2*>(lut), N, total, reinterpret_cast<uint2*>(cells));
    else
        hipLaunchKernelGGL(k_lut_to_cells<float4>, dim3((unsigned)blocks), dim3(256), 0, stream,
                           reinterpret_cast<const float4*>(lut), N, total, reinterpret_cast<float4*>(cells));
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

// Bad-query counter: the validity test of locate() (finite components, a
// nonzero major axis) per direction, summed per wavefront by ballot and
// added with one 64-bit integer atomic.
__global__ void k_count_invalid(const float* __restrict__ dirs, int64_t Q, unsigned long long* __restrict__ count)
{
    int n = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < Q; q += stride) {
        const float x = dirs[3 * q], y = dirs[3 * q + 1], z = dirs[3 * q + 2];
        const float ma = fmaxf(fabsf(x), fmaxf(fabsf(y), fabsf(z)));
        n += (isfinite(x) && isfinite(y) && isfinite(z) && ma > 0.0f) ? 0 : 1;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) n += __shfl_xor(n, o, 64);
    if ((threadIdx.x & 63) == 0 && n > 0) atomicAdd(count, (unsigned long long)n);
}

int launch_count_invalid(const float* dirs, int64_t Q, unsigned long long* count, hipStream_t stream)
{
    if (Q == 0) return SHM_OK;
    const int64_t blocks = std::min<int64_t>((Q + 255) / 256, 4096);
    hipLaunchKernelGGL(k_count_invalid, dim3((unsigned)blocks), dim3(256), 0, stream, dirs, Q, count);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

}  // namespace shm
