// Pieces of the fitting step (the differentiation form) shared by its
// separate kernels and the fused step kernel: the gradient of the value +
// normal objective with respect to one query's output, one Adam update of
// one parameter, and the host-side Adam constants.
#pragma once
#include <cmath>
#include <cstdint>

#include <hip/hip_runtime.h>

#include "shm_device.hpp"

namespace shm {

// L = w_value mean_q (R_q - R*_q)^2 + mean_q |n_q - n*_q|^2 with
// n = (R w - g) / |R w - g| (Eq. 10), w = d/|d|.  With m = R w - g:
// d|n - n*|^2/dm = (2/|m|) (e - n (n.e)), e = n - n*; dm/dR = w and
// dm/dg = -I.  Queries whose output is not finite (zero or non-finite
// directions) or whose m vanishes contribute nothing.  The reciprocal
// square roots are the hardware's (~1 ulp): a gradient, no decision.
__device__ __forceinline__ float4 loss_grad_one(float4 o, float dx, float dy, float dz, float tr, float tnx,
                                                float tny, float tnz, float w_value, float inv_q)
{
    const float3 w = unit_dir(dx, dy, dz);
    const float wx = w.x, wy = w.y, wz = w.z;
    const float mx = o.x * wx - o.y, my = o.x * wy - o.z, mz = o.x * wz - o.w;
    const float ml2 = mx * mx + my * my + mz * mz;
    float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
    if (isfinite(o.x) && isfinite(ml2) && ml2 > 0.0f) {
        const float im = __builtin_amdgcn_rsqf(ml2);
        const float nx = mx * im, ny = my * im, nz = mz * im;
        const float ex = nx - tnx, ey = ny - tny, ez = nz - tnz;
        const float ne = nx * ex + ny * ey + nz * ez;
        const float c = 2.0f * inv_q * im;
        const float gmx = c * (ex - nx * ne), gmy = c * (ey - ny * ne), gmz = c * (ez - nz * ne);
        g.x = 2.0f * w_value * inv_q * (o.x - tr) + (gmx * wx + gmy * wy + gmz * wz);
        g.y = -gmx;
        g.z = -gmy;
        g.w = -gmz;
    }
    return g;
}

// The forward query inside the fitting step, from a located valid
// direction: the plain query's patch arithmetic with the hardware square
// root in the chart-to-sphere transport (the cell decision stays the exact
// one: the backward's query lists are built from it).
__device__ __forceinline__ float4 fit_forward(const float* __restrict__ lut, int N, const Loc& L)
{
    const Foot F = load_foot<false, false>(lut, N, L);
    const Patch P = hermite(F, L.s, L.t);
    const float Nf = (float)N;
    const float3 g = transport_t<true>(L.face, L.a, L.b, Nf * P.rs, Nf * P.rt);
    return make_float4(P.r, g.x, g.y, g.z);
}

// Adam in the form PyTorch applies it: m <- m + (1 - b1)(g - m),
// v <- b2 v + (1 - b2) g^2, p <- p - (lr / bc1) m / (sqrt(v) / sqrt(bc2) + eps)
// with bc1 = 1 - b1^t, bc2 = 1 - b2^t.  The square root and the reciprocal
// are the hardware's (~1 ulp each), so the update is within a few ulps of
// that form.
struct AdamConsts {
    float step_value, step_deriv;  // lr / bc1 for channel 0 and channels 1..3
    float b1, b2, inv_bc2_sqrt, eps;
};

// Bias corrections in double, as the reference optimiser forms them.
inline AdamConsts adam_consts(int64_t step, float lr_value, float lr_deriv, float b1, float b2, float eps)
{
    const double bc1 = 1.0 - std::pow((double)b1, (double)step);
    const double bc2 = 1.0 - std::pow((double)b2, (double)step);
    return AdamConsts{(float)(lr_value / bc1), (float)(lr_deriv / bc1), b1, b2, (float)(1.0 / std::sqrt(bc2)), eps};
}

__device__ __forceinline__ void adam1(float& p, float g, float& m, float& v, float step, const AdamConsts& k)
{
    m = m + (1.0f - k.b1) * (g - m);
    v = k.b2 * v + (1.0f - k.b2) * g * g;
    p = p - step * m * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(v) * k.inv_bc2_sqrt + k.eps);
}

// One texel (r, r_u h, r_v h, r_uv h^2): the value channel with its own rate.
__device__ __forceinline__ void adam_texel(float4& p, float4 g, float4& m, float4& v, const AdamConsts& k)
{
    adam1(p.x, g.x, m.x, v.x, k.step_value, k);
    adam1(p.y, g.y, m.y, v.y, k.step_deriv, k);
    adam1(p.z, g.z, m.z, v.z, k.step_deriv, k);
    adam1(p.w, g.w, m.w, v.w, k.step_deriv, k);
}

}  // namespace shm
