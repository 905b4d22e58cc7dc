// Ray casting against the star-shaped surface x(w) = c + R(w) w (Sec. 3.1).
//
// One lane per ray.  Every evaluation of F(t) = |p - c| - R(w) is a full
// Hermite query (locate, 16-scalar gather, patch, closed-form gradient), so
// F'(t) = d.w - (d . grad R)/|p - c| comes from the same four texels.
// Schedule, the same as the oracle's: bounding sphere -> uniform march to
// the first F < 0 -> bisection -> safeguarded Newton -> final evaluation.
// Fixed iteration counts keep the FP32 path on the same steps as an FP64
// evaluation of the same schedule.  R is the rendered radius: s r, or s |r|
// for a signed function.  Optionally the number of bisections adapts to the
// glyph's projected size (Sec. 3.1), decided per ray in FP32.
#include "shm_device.hpp"
#include "shm_internal.hpp"

namespace shm {

struct FEval {
    float F, dF, R;
    float3 g, w;
    int sgn;
};

// FAST evaluations (the iterations) use the hardware reciprocal, square
// root and reciprocal square root (~1 ulp each) instead of the correctly
// rounded sequences; the final evaluation, whose R, gradient and normal are
// returned, is the exact query.
template <bool FP16, bool CELL, bool FAST = true>
__device__ __forceinline__ FEval trace_eval(const void* __restrict__ lut, int N, float ox, float oy, float oz,
                                            float dx, float dy, float dz, float t, float scale, bool is_signed)
{
    FEval E;
    const float px = ox + t * dx, py = oy + t * dy, pz = oz + t * dz;
    const float4 r = rendered(query_one<FP16, CELL, FAST>(lut, N, px, py, pz), scale, is_signed, &E.sgn);
    const float p2 = px * px + py * py + pz * pz;
    const float il = FAST ? __builtin_amdgcn_rsqf(p2) : 1.0f / sqrtf(p2);
    const float len = FAST ? p2 * il : sqrtf(p2);
    E.R = r.x;
    E.g = make_float3(r.y, r.z, r.w);
    E.w = make_float3(px * il, py * il, pz * il);
    E.F = len - r.x;
    E.dF = (dx * E.w.x + dy * E.w.y + dz * E.w.z) - (dx * r.y + dy * r.z + dz * r.w) * il;
    return E;
}

// Empty-space test of a march sample against the block bound map (map
// [6][B][B], bounds of r from the cells' Bezier control points): true when
// |p - c| exceeds scale * bound (with a 2^-12 margin, far above the
// rounding of the bound, of |p - c| and of the evaluated R), so F > 0 there
// and the evaluation that would say so can be skipped.  The face is chosen
// as the query chooses it; the block from a hardware-reciprocal (u, v),
// which the map's one-cell widening covers.
__device__ __forceinline__ bool outside_bound(const float* __restrict__ map, int B, float scale, float x, float y,
                                              float z)
{
    const float ax = fabsf(x), ay = fabsf(y), az = fabsf(z);
    const bool isx = (ax >= ay) && (ax >= az);
    const bool isy = !isx && (ay >= az);
    float sc, tc, ma;
    int face;
    if (isx) {
        const bool pos = x >= 0.0f;
        face = pos ? 0 : 1;
        ma = ax;
        sc = pos ? -z : z;
        tc = -y;
    } else if (isy) {
        const bool pos = y >= 0.0f;
        face = pos ? 2 : 3;
        ma = ay;
        sc = x;
        tc = pos ? z : -z;
    } else {
        const bool pos = z >= 0.0f;
        face = pos ? 4 : 5;
        ma = az;
        sc = pos ? x : -x;
        tc = -y;
    }
    if (!(ma > 0.0f) || !(ma < __builtin_inff())) return false;
    const float rm = __builtin_amdgcn_rcpf(ma);
    const float Bf = (float)B;
    int bi = (int)((sc * rm + 1.0f) * 0.5f * Bf), bj = (int)((tc * rm + 1.0f) * 0.5f * Bf);
    bi = bi < 0 ? 0 : (bi >= B ? B - 1 : bi);
    bj = bj < 0 ? 0 : (bj >= B ? B - 1 : bj);
    const float rb = scale * map[(face * B + bj) * B + bi] * (1.0f + 1.0f / 4096.0f);
    return x * x + y * y + z * z > rb * rb;
}

// Bisection budget: the march bracket (at most 2 rmax / n_march long) spans
// e = 2 rmax px / (|o - c| n_march) pixels at the glyph's depth, px being
// the focal length in pixels; halve until e <= eps_px, at most n_bisect
// times.  Every step is rounded to nearest without contraction (halving is
// exact), the order fixed, so the count is reproducible bit for bit.
__device__ __noinline__ int bisect_budget(float ox, float oy, float oz, float rmax, float px, float eps_px, int n_march,
                                          int n_bisect)
{
#pragma clang fp contract(off)
    const float dd = ox * ox + oy * oy + oz * oz;
    const float depth = sqrtf(dd);
    float e = (2.0f * rmax * px) / (depth * (float)n_march);
    int k = 0;
    while (k < n_bisect && e > eps_px) {
        e *= 0.5f;
        ++k;
    }
    return k;
}

template <bool FP16, bool CELL, bool NRM>
__global__ __launch_bounds__(256) void k_trace(const void* __restrict__ lut, int N, float cx, float cy, float cz,
                                               float rmax, float scale, int is_signed_i, float px_focal, float eps_px,
                                               const float* __restrict__ ray_o, const float* __restrict__ ray_d,
                                               int64_t P, int img_w, int64_t tiles_x,
                                               const float* __restrict__ bmap, int bmap_b, int n_march,
                                               int n_bisect_max, int n_newton, float* __restrict__ t_out,
                                               float* __restrict__ out, float* __restrict__ nrm,
                                               int8_t* __restrict__ sign_out, uint8_t* __restrict__ evals_out)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (img_w > 0) {
        // wavefront -> 8 x 8 pixel tile of the row-major image (tiles row by
        // row), lane -> pixel in the tile; pixels past the right or bottom
        // edge have no ray
        const int64_t tile = r >> 6;
        const int lane = (int)(r & 63);
        const int64_t ty = tile / tiles_x, tx = tile - ty * tiles_x;
        const int64_t x = tx * 8 + (lane & 7), y = ty * 8 + (lane >> 3);
        if (x >= img_w) return;
        r = y * img_w + x;
    }
    if (r >= P) return;
    const bool is_signed = is_signed_i != 0;
    // origin relative to the centre; unit direction
    const float ox = ray_o[3 * r] - cx, oy = ray_o[3 * r + 1] - cy, oz = ray_o[3 * r + 2] - cz;
    const int n_bisect =
        px_focal > 0.0f ? bisect_budget(ox, oy, oz, rmax, px_focal, eps_px, n_march, n_bisect_max) : n_bisect_max;
    int evals = 0;
    float dx = ray_d[3 * r], dy = ray_d[3 * r + 1], dz = ray_d[3 * r + 2];
    const float dl = sqrtf(dx * dx + dy * dy + dz * dz);
    dx /= dl;
    dy /= dl;
    dz /= dl;
    // disc = rmax^2 - (squared distance of the centre from the ray line),
    // formed from the perpendicular vector: b^2 - (|o - c|^2 - rmax^2)
    // cancels catastrophically in FP32 once |o - c| >> rmax
    const float b = ox * dx + oy * dy + oz * dz;
    const float hx = ox - b * dx, hy = oy - b * dy, hz = oz - b * dz;
    const float disc = rmax * rmax - (hx * hx + hy * hy + hz * hz);
    bool hit = false;
    float t = __builtin_inff();
    if (disc >= 0.0f && dl > 0.0f) {
        const float sq = sqrtf(disc);
        const float tin = -b - sq, tout = -b + sq;
        if (tout >= 0.0f) {
            const float t0 = tin > 0.0f ? tin : 0.0f, t1 = tout;
            const float step = (t1 - t0) / (float)n_march;
            float lo = t0, hi = t0;
            for (int k = 1; k <= n_march; ++k) {
                const float tk = t0 + (float)k * step;
                if (bmap && outside_bound(bmap, bmap_b, scale, ox + tk * dx, oy + tk * dy, oz + tk * dz))
                    continue;  // F > 0 there for certain: the march goes on, as it would after evaluating
                const FEval E = trace_eval<FP16, CELL>(lut, N, ox, oy, oz, dx, dy, dz, tk, scale, is_signed);
                ++evals;
                if (E.F < 0.0f) {
                    hit = true;
                    lo = t0 + (float)(k - 1) * step;
                    hi = tk;
                    break;
                }
            }
            if (hit) {
                for (int it = 0; it < n_bisect; ++it) {
                    const float mid = 0.5f * (lo + hi);
                    const FEval E = trace_eval<FP16, CELL>(lut, N, ox, oy, oz, dx, dy, dz, mid, scale, is_signed);
                    ++evals;
                    if (E.F < 0.0f) hi = mid;
                    else lo = mid;
                }
                t = 0.5f * (lo + hi);
                for (int it = 0; it < n_newton; ++it) {
                    const FEval E = trace_eval<FP16, CELL>(lut, N, ox, oy, oz, dx, dy, dz, t, scale, is_signed);
                    ++evals;
                    if (E.F < 0.0f) hi = t;
                    else lo = t;
                    float tn = t - E.F * __builtin_amdgcn_rcpf(E.dF);
                    if (!(tn >= lo && tn <= hi)) tn = 0.5f * (lo + hi);
                    t = tn;
                }
            }
        }
    }
    if (hit) {
        const FEval E = trace_eval<FP16, CELL, false>(lut, N, ox, oy, oz, dx, dy, dz, t, scale, is_signed);
        ++evals;
        if (sign_out) sign_out[r] = (int8_t)E.sgn;
        t_out[r] = t;
        reinterpret_cast<float4*>(out)[r] = make_float4(E.R, E.g.x, E.g.y, E.g.z);
        if constexpr (NRM) {
            const float mx = E.R * E.w.x - E.g.x, my = E.R * E.w.y - E.g.y, mz = E.R * E.w.z - E.g.z;
            const float in = rsqrtf(mx * mx + my * my + mz * mz);
            nrm[3 * r] = mx * in;
            nrm[3 * r + 1] = my * in;
            nrm[3 * r + 2] = mz * in;
        }
    } else {
        const float nan = __builtin_nanf("");
        if (sign_out) sign_out[r] = 0;
        t_out[r] = __builtin_inff();
        reinterpret_cast<float4*>(out)[r] = make_float4(nan, nan, nan, nan);
        if constexpr (NRM) {
            nrm[3 * r] = nan;
            nrm[3 * r + 1] = nan;
            nrm[3 * r + 2] = nan;
        }
    }
    if (evals_out) evals_out[r] = (uint8_t)evals;
}

int launch_trace(const void* lut, int dtype, int N, const float* center, float rmax, float scale, int flags,
                 float px_focal, float eps_px, const float* ray_o, const float* ray_d, int64_t P, int image_width,
                 const float* bound_map, int bound_blocks, int n_march, int n_bisect, int n_newton, float* t_out,
                 float* out, float* normal, int8_t* sign, uint8_t* evals, hipStream_t stream)
{
    if (P == 0) return SHM_OK;
    // one lane per ray, or (image rays) one wavefront per 8 x 8 tile
    int64_t tiles_x = 0, lanes = P;
    if (image_width > 0) {
        const int64_t h = P / image_width;
        tiles_x = ((int64_t)image_width + 7) / 8;
        lanes = tiles_x * ((h + 7) / 8) * 64;
    }
    const int64_t blocks = (lanes + 255) / 256;
    if (blocks > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "trace: too many rays");
    const dim3 g((unsigned)blocks), bl(256);
    const float cx = center[0], cy = center[1], cz = center[2];
    const int sgn = (flags & SHM_SIGNED) ? 1 : 0;
    const bool cell = (flags & SHM_CELL_LUT) != 0;
#define SHM_T(F, C, NR)                                                                                               \
    hipLaunchKernelGGL((k_trace<F, C, NR>), g, bl, 0, stream, lut, N, cx, cy, cz, rmax, scale, sgn, px_focal, eps_px,   \
                       ray_o, ray_d, P, image_width, tiles_x, bound_blocks > 0 ? bound_map : nullptr, bound_blocks,   \
                       n_march, n_bisect, n_newton, t_out, out, normal, sign, evals)
    if (dtype == SHM_F16) {
        if (cell) { if (normal) SHM_T(true, true, true); else SHM_T(true, true, false); }
        else { if (normal) SHM_T(true, false, true); else SHM_T(true, false, false); }
    } else {
        if (cell) { if (normal) SHM_T(false, true, true); else SHM_T(false, true, false); }
        else { if (normal) SHM_T(false, false, true); else SHM_T(false, false, false); }
    }
#undef SHM_T
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

}  // namespace shm
