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
