/*
 * shm_probe.h -- memory-system probes of libshm (measurement, not part of
 * the method).
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
 * 64 or 128) at the aligned offset req_bytes * floor(h(r) * S / 2^32) of
 * its region, S = floor(region_bytes / req_bytes), h a 32-bit integer hash
 * of (seed, r); one lane per request, 256 requests of one region per
 * workgroup (the query's launch mapping).
 *   base          n_regions * region_bytes readable bytes, 16-byte aligned;
 *                 region_bytes a multiple of 16 and >= req_bytes
 *   dirs          NULL: gathers only, and out is a 16-byte sink that is not
 *                 written for finite data;  non-NULL: [n_regions *
 *                 per_region][3] FP32 streamed as the query streams its
 *                 directions, and out [n_regions * per_region][4] FP32 (16-byte
 *                 aligned) receives one 16 B result per request, as the
 *                 query writes its results
 * Errors: SHM_ERR_INVALID_ARG for a bad size, alignment or null pointer. */
SHM_API int shm_probe_gather(const void* base, int64_t region_bytes, int64_t n_regions, int64_t per_region,
                             int32_t req_bytes, uint32_t seed, const float* dirs, float* out, hipStream_t stream);

/* Streaming read of `bytes` bytes (a multiple of 16) at base (16-byte
 * aligned); sink is a 16-byte buffer that is not written for finite data. */
SHM_API int shm_probe_stream_read(const void* base, int64_t bytes, float* sink, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SHM_PROBE_H */
