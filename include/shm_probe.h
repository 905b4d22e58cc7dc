/*
 * shm_probe.h -- memory-system and matrix-core probes of libshm
 * (measurement, not part of the method).
 *
 * The value + gradient query of Spherical Hermite Maps reads, per query, the
 * 2x2 texel footprint of its cell (16 scalars, Sec. 3.3 Eq. 4 and Table
 * cost_extended) plus its direction, and writes its result.  In the CELL
 * layout the footprint is one aligned 64 B (FP32) block at a data-dependent
 * place inside the object's LUT.  These probes issue that traffic without
 * the arithmetic, so the query's throughput can be set against what the
 * memory system delivers for the same access pattern.  Same conventions as
 * shm.h: device pointers, asynchronous on `stream`, host-side validation,
 * status codes, no allocation.
 */
#ifndef SHM_PROBE_H
#define SHM_PROBE_H

#include "shm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Random gathers inside regions.  Request r (0 <= r < n_regions *
 * per_region) belongs to region r / per_region and reads req_bytes (16, 32,
 * 64 or 128; 0 reads nothing) at the aligned offset req_bytes * floor(h(r) *
 * S / 2^32) of its region, S = floor(region_bytes / req_bytes), h a 32-bit
 * integer hash of (seed, r); one lane per request, 256 requests of one
 * region per workgroup (the query's launch mapping).  flags:
 *   SHM_PROBE_DIRS  also read the request's direction dirs[r][0..2] (FP32)
 *                   as the query streams its directions
 *   SHM_PROBE_OUT   also write one 16 B result per request to out[r][0..3]
 *                   (FP32), as the query writes its results
 *   base    n_regions * region_bytes readable bytes, 16-byte aligned (unused
 *           when req_bytes is 0); region_bytes a multiple of 16, >= req_bytes
 *   dirs    [n_regions * per_region][3] with SHM_PROBE_DIRS, else unused
 *   out     [n_regions * per_region][4], 16-byte aligned, with SHM_PROBE_OUT;
 *           else a 16-byte sink that is not written for finite data
 * Errors: SHM_ERR_INVALID_ARG for a bad size, flag, alignment or null
 * pointer. */
#define SHM_PROBE_DIRS 1
#define SHM_PROBE_OUT 2
SHM_API int shm_probe_gather(const void* base, int64_t region_bytes, int64_t n_regions, int64_t per_region,
                             int32_t req_bytes, uint32_t seed, int32_t flags, const float* dirs, float* out,
                             hipStream_t stream);

/* Streaming read of `bytes` bytes (a multiple of 16) at base (16-byte
 * aligned); sink is a 16-byte buffer that is not written for finite data. */
SHM_API int shm_probe_stream_read(const void* base, int64_t bytes, float* sink, hipStream_t stream);

/* The FP32 matrix cores without memory traffic: waves_per_simd (1..8)
 * workgroups of 4 waves per compute unit, each wave running `iters` (>= 1)
 * rounds of `chains` (1, 2, 4 or 8) independent v_mfma_f32_16x16x4f32 on
 * register operands, 2,048 flops each; the bake's contraction (Sec. 3.3,
 * the basis x coefficient product) uses the same instruction.  *flops
 * (host pointer) receives the launch's flop count before the launch; sink
 * is a 16-byte aligned device buffer that is not written for finite data.
 * Errors: SHM_ERR_INVALID_ARG for an argument out of range or a null or
 * misaligned pointer. */
SHM_API int shm_probe_mfma_f32(int32_t waves_per_simd, int32_t chains, int64_t iters, double* flops, float* sink,
                               hipStream_t stream);

/* The batched form's memory traffic without its arithmetic: the walk of
 * shm_plan_launch over the plan's work list, in the plan's current launch
 * shape, where each query q reads its direction dirs[q][0..2], the
 * footprint of one pseudo-random cell of its object's LUT (cell index
 * floor(h(q) * 6 (N+1)^2 / 2^32), h a 32-bit integer hash of (seed, q);
 * loaded as the query loads it in the plan's dtype and layout: one 64 B
 * (FP32) or 32 B (FP16) block in the CELL layout, two rows of two texels in
 * the TEXEL layout), and writes out[q] = (dirs[q][0..2], w) with w the
 * 32-bit pattern of the wrapping sum of the footprint's 32-bit words.
 * Arguments as for shm_plan_launch (lut, dirs, out of the plan's objects;
 * out 16-byte aligned, lut 16-byte aligned, 8 for FP16 texels).  The launch
 * counts as a launch of the plan (shm_plan_set_shape and
 * shm_plan_destroy wait for it).
 * Errors: SHM_ERR_INVALID_ARG for a null plan or pointer or a misaligned
 * buffer. */
SHM_API int shm_plan_probe(shm_plan* plan, const void* lut, const float* dirs, float* out, uint32_t seed,
                           hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SHM_PROBE_H */
