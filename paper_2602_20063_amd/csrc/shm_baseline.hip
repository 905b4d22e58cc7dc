// Comparison paths of the paper's experiments (Sec. 4.2, 4.5, 4.6), run on the
// same GPU as the Hermite query:
//   * value-only LUT reconstructions (Table cost_extended, Table runtime):
//     nearest texel, bilinear with finite-difference normals (4 extra
//     bilinear lookups at u +- h, v +- h), 16-tap Catmull-Rom bicubic with its
//     analytic gradient, and "fast bicubic": the cubic B-spline (what four
//     hardware-bilinear fetches evaluate), with the same finite-difference
//     gradient.  Without texture units every method but nearest reads the
//     4 x 4 texel footprint of its cell once into registers (the bilinear
//     lookups at +-1 texel fall inside it) and filters from there;
//   * direct SH evaluation without any LUT (the paper's per-fragment SH
//     baseline, Sec. 4.6).
// The value-only LUT is vlut[obj][face][q][p], p, q in 0..N+3, texel p at
// u = (p - 3/2)/N (two-texel gutter, the sample grid of shm_margin_dirs).
#include "shm_device.hpp"
#include "shm_internal.hpp"

namespace shm {

__device__ __forceinline__ float vl_at(const float* __restrict__ vl, int P, int face, int p, int q)
{
    p = p < 0 ? 0 : (p > P - 1 ? P - 1 : p);
    q = q < 0 ? 0 : (q > P - 1 ? P - 1 : q);
    return vl[((int64_t)face * P + q) * P + p];
}

template <int METHOD>
__global__ __launch_bounds__(256) void k_query_baseline(const float* __restrict__ vlut, int N, int64_t q_per_obj,
                                                        int tiles_per_obj, const float* __restrict__ dirs,
                                                        float* __restrict__ out)
{
    const int b = (int)blockIdx.x;
    const int obj = b / tiles_per_obj;
    const int64_t ql = (int64_t)(b - obj * tiles_per_obj) * 256 + threadIdx.x;
    if (ql >= q_per_obj) return;
    const int64_t q = (int64_t)obj * q_per_obj + ql;
    const int P = N + 4;
    const float* vl = vlut + (int64_t)obj * 6 * P * P;
    const float x = dirs[3 * q], y = dirs[3 * q + 1], z = dirs[3 * q + 2];
    const Loc L = locate(x, y, z, N);
    if (L.face < 0) {
        const float nan = __builtin_nanf("");
        reinterpret_cast<float4*>(out)[q] = make_float4(nan, nan, nan, nan);
        return;
    }
    const float a = L.a, bb = L.b, Nf = (float)N;
    float R, ru = 0.0f, rv = 0.0f;
    if constexpr (METHOD == SHM_RECON_NEAREST) {
        const float fu = (a + 1.0f) * 0.5f * Nf + 1.5f, fv = (bb + 1.0f) * 0.5f * Nf + 1.5f;
        R = vl_at(vl, P, L.face, (int)floorf(fu + 0.5f), (int)floorf(fv + 0.5f));
    } else {
        const float fu = (a + 1.0f) * 0.5f * Nf + 1.5f, fv = (bb + 1.0f) * 0.5f * Nf + 1.5f;
        const int i0 = (int)floorf(fu), j0 = (int)floorf(fv);
        const float s = fu - (float)i0, t = fv - (float)j0;
        float v[4][4];  // v[j][i]: texel (i0 - 1 + i, j0 - 1 + j)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) v[j][i] = vl_at(vl, P, L.face, i0 - 1 + i, j0 - 1 + j);
        if constexpr (METHOD == SHM_RECON_BICUBIC) {
            float ws[4], dws[4], wt[4], dwt[4];
            {
                const float s2 = s * s, s3 = s2 * s, t2 = t * t, t3 = t2 * t;
                ws[0] = 0.5f * (-s3 + 2.0f * s2 - s);
                ws[1] = 0.5f * (3.0f * s3 - 5.0f * s2 + 2.0f);
                ws[2] = 0.5f * (-3.0f * s3 + 4.0f * s2 + s);
                ws[3] = 0.5f * (s3 - s2);
                dws[0] = 0.5f * (-3.0f * s2 + 4.0f * s - 1.0f);
                dws[1] = 0.5f * (9.0f * s2 - 10.0f * s);
                dws[2] = 0.5f * (-9.0f * s2 + 8.0f * s + 1.0f);
                dws[3] = 0.5f * (3.0f * s2 - 2.0f * s);
                wt[0] = 0.5f * (-t3 + 2.0f * t2 - t);
                wt[1] = 0.5f * (3.0f * t3 - 5.0f * t2 + 2.0f);
                wt[2] = 0.5f * (-3.0f * t3 + 4.0f * t2 + t);
                wt[3] = 0.5f * (t3 - t2);
                dwt[0] = 0.5f * (-3.0f * t2 + 4.0f * t - 1.0f);
                dwt[1] = 0.5f * (9.0f * t2 - 10.0f * t);
                dwt[2] = 0.5f * (-9.0f * t2 + 8.0f * t + 1.0f);
                dwt[3] = 0.5f * (3.0f * t2 - 2.0f * t);
            }
            R = 0.0f;
            float rs = 0.0f, rt = 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float row = 0.0f, drow = 0.0f;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    row += ws[i] * v[j][i];
                    drow += dws[i] * v[j][i];
                }
                R += wt[j] * row;
                rs += wt[j] * drow;
                rt += dwt[j] * row;
            }
            ru = Nf * rs;
            rv = Nf * rt;
        } else {
            // bilinear lookups at the cell and one texel to either side
            auto bil = [&](int j, int i, float fx, float fy) {
                const float r0 = v[j][i] + fx * (v[j][i + 1] - v[j][i]);
                const float r1 = v[j + 1][i] + fx * (v[j + 1][i + 1] - v[j + 1][i]);
                return r0 + fy * (r1 - r0);
            };
            const float hN = 0.5f * Nf;  // 1 / (2h): central difference over +-1 texel
            ru = (bil(1, 2, s, t) - bil(1, 0, s, t)) * hN;
            rv = (bil(2, 1, s, t) - bil(0, 1, s, t)) * hN;
            if constexpr (METHOD == SHM_RECON_BILINEAR_FD) {
                R = bil(1, 1, s, t);
            } else {
                // uniform cubic B-spline weights of taps -1..2
                float ws[4], wt[4];
                {
                    const float s2 = s * s, s3 = s2 * s, ms = 1.0f - s;
                    const float t2 = t * t, t3 = t2 * t, mt = 1.0f - t;
                    const float k = 1.0f / 6.0f;
                    ws[0] = ms * ms * ms * k;
                    ws[1] = (3.0f * s3 - 6.0f * s2 + 4.0f) * k;
                    ws[2] = (-3.0f * s3 + 3.0f * s2 + 3.0f * s + 1.0f) * k;
                    ws[3] = s3 * k;
                    wt[0] = mt * mt * mt * k;
                    wt[1] = (3.0f * t3 - 6.0f * t2 + 4.0f) * k;
                    wt[2] = (-3.0f * t3 + 3.0f * t2 + 3.0f * t + 1.0f) * k;
                    wt[3] = t3 * k;
                }
                R = 0.0f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float row = 0.0f;
#pragma unroll
                    for (int i = 0; i < 4; ++i) row += ws[i] * v[j][i];
                    R += wt[j] * row;
                }
            }
        }
    }
    const float3 g = transport(L.face, a, bb, ru, rv);
    reinterpret_cast<float4*>(out)[q] = make_float4(R, g.x, g.y, g.z);
}

int launch_query_baseline(const float* vlut, int N, int64_t n_obj, const float* dirs, int64_t q_per_obj, int method,
                          float* out, hipStream_t stream)
{
    if (n_obj == 0 || q_per_obj == 0) return SHM_OK;
    const int64_t tiles = (q_per_obj + 255) / 256;
    if (tiles * n_obj > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "query_baseline: too many tiles for one launch");
    const dim3 grid((unsigned)(tiles * n_obj)), block(256);
    if (method == SHM_RECON_NEAREST)
        hipLaunchKernelGGL(k_query_baseline<SHM_RECON_NEAREST>, grid, block, 0, stream, vlut, N, q_per_obj, (int)tiles, dirs, out);
    else if (method == SHM_RECON_BILINEAR_FD)
        hipLaunchKernelGGL(k_query_baseline<SHM_RECON_BILINEAR_FD>, grid, block, 0, stream, vlut, N, q_per_obj, (int)tiles, dirs, out);
    else if (method == SHM_RECON_FAST_BICUBIC_FD)
        hipLaunchKernelGGL(k_query_baseline<SHM_RECON_FAST_BICUBIC_FD>, grid, block, 0, stream, vlut, N, q_per_obj, (int)tiles, dirs, out);
    else
        hipLaunchKernelGGL(k_query_baseline<SHM_RECON_BICUBIC>, grid, block, 0, stream, vlut, N, q_per_obj, (int)tiles, dirs, out);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

// ---------------------------------------------------------------------------
// Direct SH evaluation: R = sum_k c_k Y_k(w) and its spherical gradient, the
// tangential part of the gradient of the Cartesian polynomial form
// P_{l,+-m} = sqrt2 Qn_l^m(z) {Re, Im}(x + i y)^m at w = d/|d|.  FP32, with
// the normalised Legendre recurrence (values stay O(1)).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sh_eval(const float* __restrict__ coeffs, int L, int64_t q_per_obj,
                                                 int tiles_per_obj, const float* __restrict__ dirs,
                                                 float* __restrict__ out)
{
    const int b = (int)blockIdx.x;
    const int obj = b / tiles_per_obj;
    const int64_t ql = (int64_t)(b - obj * tiles_per_obj) * 256 + threadIdx.x;
    if (ql >= q_per_obj) return;
    const int64_t q = (int64_t)obj * q_per_obj + ql;
    const int K = (L + 1) * (L + 1);
    const float* c = coeffs + (int64_t)obj * K;
    float x = dirs[3 * q], y = dirs[3 * q + 1], z = dirs[3 * q + 2];
    const float n2 = x * x + y * y + z * z;
    if (!(n2 > 0.0f) || !isfinite(n2)) {
        const float nan = __builtin_nanf("");
        reinterpret_cast<float4*>(out)[q] = make_float4(nan, nan, nan, nan);
        return;
    }
    const float in = rsqrtf(n2);
    x *= in;
    y *= in;
    z *= in;
    const float SQ2 = 1.41421356237309515f;
    float R = 0.0f, gx = 0.0f, gy = 0.0f, gz = 0.0f;
    float Am1 = 0.0f, Bm1 = 0.0f, Am = 1.0f, Bm = 0.0f;
    float diag = 0.282094791773878143f;  // Qn_0^0
    for (int m = 0; m <= L; ++m) {
        if (m > 0) {
            Am1 = Am;
            Bm1 = Bm;
            Am = Am1 * x - Bm1 * y;
            Bm = Am1 * y + Bm1 * x;
            diag *= sqrtf((float)(2 * m + 1) / (float)(2 * m));
        }
        const float d1 = diag * sqrtf((float)(2 * m + 3) / (float)(2 * m + 2));
        float p1 = 0.0f, p2 = 0.0f, e1 = 0.0f, e2 = 0.0f;  // columns m and m+1
        for (int l = m; l <= L; ++l) {
            float q0, q1;
            if (l == m) q0 = diag;
            else {
                const float ll = (float)l, mm = (float)m;
                q0 = sqrtf((4.0f * ll * ll - 1.0f) / (ll * ll - mm * mm)) * z * p1 -
                     sqrtf(((ll - 1.0f) * (ll - 1.0f) - mm * mm) * (2.0f * ll + 1.0f) / ((2.0f * ll - 3.0f) * (ll * ll - mm * mm))) * p2;
            }
            p2 = p1;
            p1 = q0;
            if (l < m + 1) q1 = 0.0f;
            else if (l == m + 1) q1 = d1;
            else {
                const float ll = (float)l, mm = (float)(m + 1);
                q1 = sqrtf((4.0f * ll * ll - 1.0f) / (ll * ll - mm * mm)) * z * e1 -
                     sqrtf(((ll - 1.0f) * (ll - 1.0f) - mm * mm) * (2.0f * ll + 1.0f) / ((2.0f * ll - 3.0f) * (ll * ll - mm * mm))) * e2;
            }
            e2 = e1;
            e1 = q1;
            const float dq = sqrtf((float)((l + m + 1) * (l - m))) * q1;
            if (m == 0) {
                const float ck = c[l * l + l];
                R += ck * q0;
                gz += ck * dq;
            } else {
                const float cp = SQ2 * c[l * l + l + m], cn = SQ2 * c[l * l + l - m];
                const float mf = (float)m;
                R += q0 * (cp * Am + cn * Bm);
                gx += q0 * mf * (cp * Am1 + cn * Bm1);
                gy += q0 * mf * (-cp * Bm1 + cn * Am1);
                gz += dq * (cp * Am + cn * Bm);
            }
        }
    }
    const float gr = gx * x + gy * y + gz * z;  // tangential part at the unit direction
    reinterpret_cast<float4*>(out)[q] = make_float4(R, gx - gr * x, gy - gr * y, gz - gr * z);
}

int launch_sh_eval(const float* coeffs, int L, int64_t n_obj, const float* dirs, int64_t q_per_obj, float* out,
                   hipStream_t stream)
{
    if (n_obj == 0 || q_per_obj == 0) return SHM_OK;
    const int64_t tiles = (q_per_obj + 255) / 256;
    if (tiles * n_obj > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "sh_eval: too many tiles for one launch");
    hipLaunchKernelGGL(k_sh_eval, dim3((unsigned)(tiles * n_obj)), dim3(256), 0, stream, coeffs, L, q_per_obj,
                       (int)tiles, dirs, out);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

}  // namespace shm
