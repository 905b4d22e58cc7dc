// Memory-system probes: the ceilings the query is measured against.
//
// The query's traffic is one random aligned read per query (its cell) inside
// the object's LUT, a streamed 12 B direction and a streamed 16 B result.
// These kernels issue exactly that traffic without the arithmetic:
//   k_probe_gather   one lane per request; a request reads req_bytes
//                    (16, 32, 64 or 128; 0: none) at a pseudo-random aligned
//                    offset inside its region, with the query's float4
//                    loads; the launch mapping is the query's (256 requests
//                    of one region per workgroup, XCD-contiguous tiles).  On
//                    request it also streams the 12 B direction and/or writes
//                    the 16 B result of every request, as the query does:
//                    with both, the query's memory pattern, whose rate bounds
//                    the query's; the parts alone show what each costs.
//   k_probe_stream   streaming reads of a whole buffer (float4 per lane,
//                    grid-stride), the bandwidth ceiling of plain reads.
//   k_probe_mfma     FP32 matrix-core rounds with register operands only: the
//                    rate the bake's contraction is measured against.
//   k_probe_plan     the batched form's traffic: the persistent kernel's walk
//                    over a plan's work list in the plan's launch shape; per
//                    query the 12 B direction, the footprint of a
//                    pseudo-random cell of its object's LUT (loaded as the
//                    query loads it: one block in the CELL layout, two texel
//                    rows in the TEXEL layout) and the 16 B result.
// Offsets come from Wellons' "lowbias32" integer hash of (seed, request).
#include "shm_device.hpp"
#include "shm_internal.hpp"
#include "../../include/shm_probe.h"

namespace shm {

__device__ __forceinline__ uint32_t lowbias32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <int REQ, bool DIRS, bool OUT>
__global__ __launch_bounds__(256) void k_probe_gather(const char* __restrict__ base, int64_t region_bytes,
                                                      int64_t per_region, int tiles_per_region, uint32_t seed,
                                                      const float* __restrict__ dirs, float* __restrict__ out)
{
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int region = b / tiles_per_region;
    const int tile = b - region * tiles_per_region;
    const int64_t ql = (int64_t)tile * 256 + threadIdx.x;
    if (ql >= per_region) return;
    const int64_t q = (int64_t)region * per_region + ql;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (DIRS) {
        acc.x = __builtin_nontemporal_load(dirs + 3 * q);
        acc.y = __builtin_nontemporal_load(dirs + 3 * q + 1);
        acc.z = __builtin_nontemporal_load(dirs + 3 * q + 2);
    }
    if constexpr (REQ > 0) {
        // slot in [0, slots): high half of the 32 x 32-bit product (slots < 2^32)
        const uint64_t slots = (uint64_t)(region_bytes / REQ);
        const uint32_t h = lowbias32((uint32_t)q * 0x9e3779b1u ^ seed ^ (uint32_t)(q >> 32));
        const uint64_t slot = ((uint64_t)h * slots) >> 32;
        const float4* p = reinterpret_cast<const float4*>(base + (int64_t)region * region_bytes + (int64_t)slot * REQ);
#pragma unroll
        for (int k = 0; k < REQ / 16; ++k) {
            const float4 v = p[k];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
    }
    if constexpr (OUT) {
        __builtin_nontemporal_store(f32x4{acc.x, acc.y, acc.z, acc.w}, reinterpret_cast<f32x4*>(out) + q);
    } else {
        // a store the compiler cannot drop but that (for finite data) never runs
        if (__float_as_uint(acc.x + acc.y + acc.z + acc.w) == 0x7fc00001u) out[0] = acc.x;
    }
}

__global__ __launch_bounds__(256) void k_probe_stream(const float4* __restrict__ p, int64_t n4, float* __restrict__ sink)
{
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p + i));
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
    }
    if (__float_as_uint(acc.x + acc.y + acc.z + acc.w) == 0x7fc00001u) sink[0] = acc.x;
}

// pseudo-random index in [0, n) of request q (n < 2^32)
__device__ __forceinline__ uint32_t probe_pick(int64_t q, uint32_t seed, uint32_t n)
{
    const uint32_t h = lowbias32((uint32_t)q * 0x9e3779b1u ^ seed ^ (uint32_t)(q >> 32));
    return (uint32_t)(((uint64_t)h * n) >> 32);
}

// The cell (face, j0, i0) of index `cell` of a LUT of face size N, as the
// location the query's footprint loads take.
__device__ __forceinline__ Loc probe_loc(int N, uint32_t cell)
{
    const uint32_t C = (uint32_t)N + 1;
    Loc L{};
    L.face = (int)(cell / (C * C));
    const uint32_t rem = cell - (uint32_t)L.face * C * C;
    L.j0 = (int)(rem / C);
    L.i0 = (int)(rem - (uint32_t)L.j0 * C);
    return L;
}

// A loaded footprint folded into a 32-bit word sum.
__device__ __forceinline__ uint32_t raw_sum(const FootRaw<true, true>& R)
{
    return R.q[0].x + R.q[0].y + R.q[0].z + R.q[0].w + R.q[1].x + R.q[1].y + R.q[1].z + R.q[1].w;
}
__device__ __forceinline__ uint32_t raw_sum(const FootRaw<true, false>& R)
{
    uint32_t a = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) a += R.h[i].x + R.h[i].y;
    return a;
}
template <bool CELL>
__device__ __forceinline__ uint32_t raw_sum(const FootRaw<false, CELL>& R)
{
    uint32_t a = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        a += __float_as_uint(R.c[i].x) + __float_as_uint(R.c[i].y) + __float_as_uint(R.c[i].z) +
             __float_as_uint(R.c[i].w);
    return a;
}

template <bool FP16, bool CELL, int QPT>
__global__ void k_probe_plan(const void* __restrict__ lut, const shm_object* __restrict__ objs,
                             const WorkItem* __restrict__ items, XcdSplit split, const float* __restrict__ dirs,
                             float* __restrict__ out, uint32_t seed)
{
    // the walk of k_query_persistent: nx groups of blocks, group x walks
    // slices x, x + nx, ... of the work list
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
        const uint32_t n_cells = 6u * (uint32_t)(N + 1) * (uint32_t)(N + 1);
        const char* base = reinterpret_cast<const char*>(lut) + (size_t)o.lut_offset * (FP16 ? 2 : 4);
        // the structure of k_query_persistent, its loads in the same order:
        // the directions, then (after them, as the query needs the direction
        // to find its cell) the footprints
        if constexpr (QPT == 1) {
            for (int k0 = 0; k0 < it.n; k0 += B) {
                const int k = k0 + (int)threadIdx.x;
                if (k >= it.n) continue;
                const int64_t q = it.q0 + k;
                float dx = __builtin_nontemporal_load(dirs + 3 * q);
                float dy = __builtin_nontemporal_load(dirs + 3 * q + 1);
                float dz = __builtin_nontemporal_load(dirs + 3 * q + 2);
                asm volatile("" : "+v"(dx), "+v"(dy), "+v"(dz));
                const FootRaw<FP16, CELL> F = load_raw<FP16, CELL>(base, N, probe_loc(N, probe_pick(q, seed, n_cells)));
                __builtin_nontemporal_store(f32x4{dx, dy, dz, __uint_as_float(raw_sum(F))},
                                            reinterpret_cast<f32x4*>(out) + q);
            }
            continue;
        }
        // QPT > 1: every load of the lane's QPT queries issued before any
        // use, no branch, results stored through a buffer range of the
        // item's it.n rows (idle lanes' stores dropped)
        const __amdgpu_buffer_rsrc_t ro =
            __builtin_amdgcn_make_buffer_rsrc(out + 4 * it.q0, (short)0, it.n * 16, 0x00020000);
        for (int k0 = 0; k0 < it.n; k0 += B * QPT) {
            float dx[QPT], dy[QPT], dz[QPT];
            FootRaw<FP16, CELL> F[QPT];
#pragma unroll
            for (int j = 0; j < QPT; ++j) {
                const int k = k0 + j * B + (int)threadIdx.x;
                const int64_t q = it.q0 + (k < it.n ? k : 0);
                dx[j] = __builtin_nontemporal_load(dirs + 3 * q);
                dy[j] = __builtin_nontemporal_load(dirs + 3 * q + 1);
                dz[j] = __builtin_nontemporal_load(dirs + 3 * q + 2);
            }
#pragma unroll
            for (int j = 0; j < QPT; ++j) asm volatile("" : "+v"(dx[j]), "+v"(dy[j]), "+v"(dz[j]));
#pragma unroll
            for (int j = 0; j < QPT; ++j)
                F[j] = load_raw<FP16, CELL>(base, N, probe_loc(N, probe_pick(it.q0 + k0 + j * B + (int)threadIdx.x,
                                                                             seed, n_cells)));
#pragma unroll
            for (int j = 0; j < QPT; ++j) pin(F[j]);
#pragma unroll
            for (int j = 0; j < QPT; ++j) {
                const uint32_t k = (uint32_t)(k0 + j * B + (int)threadIdx.x);
                const u32x4 w = {__float_as_uint(dx[j]), __float_as_uint(dy[j]), __float_as_uint(dz[j]), raw_sum(F[j])};
                __builtin_amdgcn_raw_buffer_store_b128(w, ro, k * 16u, 0, 2);
            }
        }
    }
}

int launch_probe_plan(const void* lut, int dtype, int layout, const shm_object* objs_dev, const WorkItem* items_dev,
                      int64_t n_items, const XcdSplit& split, const shm_launch_shape& shape, int n_cu,
                      const float* dirs, float* out, uint32_t seed, hipStream_t stream)
{
    if (n_items == 0) return SHM_OK;
    // grid_per_cu 0: one workgroup per work item (each runs its item and
    // exits: no store of one item waits behind the loads of the next)
    const int64_t G = plan_grid(shape, n_cu, n_items, split);
    const dim3 grid((unsigned)G), block((unsigned)shape.block);
    const bool f16 = dtype == SHM_F16, cell = layout == SHM_LAYOUT_CELL;
#define SHM_PP(F, C, Q) hipLaunchKernelGGL((k_probe_plan<F, C, Q>), grid, block, 0, stream, lut, objs_dev, items_dev, \
                                           split, dirs, out, seed)
#define SHM_PPQ(F, C)                                    \
    switch (shape.qpt) {                                 \
        case 1: SHM_PP(F, C, 1); break;                  \
        case 2: SHM_PP(F, C, 2); break;                  \
        default: SHM_PP(F, C, 4); break;                 \
    }
    if (f16) {
        if (cell) { SHM_PPQ(true, true) } else { SHM_PPQ(true, false) }
    } else {
        if (cell) { SHM_PPQ(false, true) } else { SHM_PPQ(false, false) }
    }
#undef SHM_PPQ
#undef SHM_PP
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

int launch_probe_gather(const void* base, int64_t region_bytes, int64_t n_regions, int64_t per_region, int req_bytes,
                        uint32_t seed, int flags, const float* dirs, float* out, hipStream_t stream)
{
    const int64_t tiles = (per_region + 255) / 256;
    const dim3 grid((unsigned)(tiles * n_regions));
    const char* b = reinterpret_cast<const char*>(base);
    const int tpr = (int)tiles;
    const bool d = (flags & SHM_PROBE_DIRS) != 0, o = (flags & SHM_PROBE_OUT) != 0;
#define SHM_PG3(R, D, O) hipLaunchKernelGGL((k_probe_gather<R, D, O>), grid, dim3(256), 0, stream, b, region_bytes, \
                                            per_region, tpr, seed, dirs, out)
#define SHM_PG(R)                                    \
    case R:                                          \
        if (d && o) SHM_PG3(R, true, true);          \
        else if (d) SHM_PG3(R, true, false);         \
        else if (o) SHM_PG3(R, false, true);         \
        else SHM_PG3(R, false, false);               \
        break;
    switch (req_bytes) {
        SHM_PG(0)
        SHM_PG(16)
        SHM_PG(32)
        SHM_PG(64)
        SHM_PG(128)
        default:
            return fail(SHM_ERR_INVALID_ARG, "probe_gather: req_bytes must be 0, 16, 32, 64 or 128");
    }
#undef SHM_PG
#undef SHM_PG3
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

// The FP32 matrix cores with register operands only: CH independent
// accumulator chains per wave, `iters` rounds; nothing but the MFMAs and the
// loop runs, so the launch measures the rate the matrix pipes sustain at the
// clock they hold under this load.
template <int CH>
__global__ __launch_bounds__(256) void k_probe_mfma(int64_t iters, float* __restrict__ sink)
{
    const int lane = threadIdx.x & 63;
    const float a = 1.0f + 1e-3f * (float)lane, b = 1.0f - 1e-3f * (float)lane;
    f32x4 acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
    }
    float t = 0.0f;
#pragma unroll
    for (int c = 0; c < CH; ++c) t += acc[c].x + acc[c].y + acc[c].z + acc[c].w;
    if (__float_as_uint(t) == 0x7fc00001u) sink[0] = t;  // never for finite data
}

int launch_probe_mfma(int waves_per_simd, int chains, int64_t iters, double* flops, float* sink, hipStream_t stream)
{
    // one workgroup of 4 waves (one per SIMD) per compute unit and wave slot
    const int64_t groups = (int64_t)device_cu_count() * waves_per_simd;
    *flops = (double)groups * 4 * iters * chains * 2.0 * 16 * 16 * 4;
    const dim3 grid((unsigned)groups), block(256);
    switch (chains) {
        case 1: hipLaunchKernelGGL(k_probe_mfma<1>, grid, block, 0, stream, iters, sink); break;
        case 2: hipLaunchKernelGGL(k_probe_mfma<2>, grid, block, 0, stream, iters, sink); break;
        case 4: hipLaunchKernelGGL(k_probe_mfma<4>, grid, block, 0, stream, iters, sink); break;
        default: hipLaunchKernelGGL(k_probe_mfma<8>, grid, block, 0, stream, iters, sink); break;
    }
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

int launch_probe_stream(const void* base, int64_t bytes, float* sink, hipStream_t stream)
{
    const int64_t n4 = bytes / 16;
    const int64_t blocks = std::min<int64_t>((n4 + 255) / 256, (int64_t)device_cu_count() * 32);
    hipLaunchKernelGGL(k_probe_stream, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, stream,
                       reinterpret_cast<const float4*>(base), n4, sink);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

}  // namespace shm
