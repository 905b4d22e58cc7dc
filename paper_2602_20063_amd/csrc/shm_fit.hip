// Fitting a map to a target (the differentiation form): the two steps of the
// optimisation loop around the query and its backward, so that a whole step
// (forward, loss gradient, backward, update) runs in this library's kernels
// and can be captured in one graph.
//
//   k_fit_loss_grad: dL/d(R, grad R) of the value + normal objective
//     L = w_value mean_q (R_q - R*_q)^2 + mean_q |n_q - n*_q|^2,
//     n = (R w - grad R) / |R w - grad R| (Eq. 10), one lane per query;
//   k_fit_forward_loss_grad: the forward query fused with it;
//   k_adam: one Adam update of the LUT (one learning rate for the value
//     channel, one for the three scaled derivative channels), one lane per
//     texel (float4).
#include <cmath>

#include "shm_device.hpp"
#include "shm_internal.hpp"

namespace shm {

// With m = R w - g and n = m/|m|: d|n - n*|^2/dm = (2/|m|) (e - n (n.e)),
// e = n - n*; dm/dR = w and dm/dg = -I.  Queries whose output is not finite
// (zero or non-finite directions) or whose m vanishes contribute nothing.
__device__ __forceinline__ float4 loss_grad_one(float4 o, float dx, float dy, float dz, float tr, float tnx,
                                                float tny, float tnz, float w_value, float inv_q)
{
    const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    const float wx = dx * il, wy = dy * il, wz = dz * il;
    const float mx = o.x * wx - o.y, my = o.x * wy - o.z, mz = o.x * wz - o.w;
    const float ml = sqrtf(mx * mx + my * my + mz * mz);
    float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
    if (isfinite(o.x) && isfinite(ml) && ml > 0.0f) {
        const float im = 1.0f / ml;
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

__global__ void k_fit_loss_grad(const float4* __restrict__ out, const float* __restrict__ dirs,
                                const float* __restrict__ tr, const float* __restrict__ tn, int64_t Q, float w_value,
                                float inv_q, float4* __restrict__ grad)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    grad[q] = loss_grad_one(out[q], dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2], tr[q], tn[3 * q], tn[3 * q + 1],
                            tn[3 * q + 2], w_value, inv_q);
}

// The forward query of a FP32 TEXEL LUT fused with the loss gradient: the
// same query arithmetic as the plain forward (so the same bits), without
// writing (R, grad R) out and reading it back.
__global__ void k_fit_forward_loss_grad(const float* __restrict__ lut, int N, const float* __restrict__ dirs,
                                        const float* __restrict__ tr, const float* __restrict__ tn, int64_t Q,
                                        float w_value, float inv_q, float4* __restrict__ grad)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    const float x = dirs[3 * q], y = dirs[3 * q + 1], z = dirs[3 * q + 2];
    const float4 o = query_one<false, false>(lut, N, x, y, z);
    grad[q] = loss_grad_one(o, x, y, z, tr[q], tn[3 * q], tn[3 * q + 1], tn[3 * q + 2], w_value, inv_q);
}

// Adam in the form PyTorch applies it: m <- m + (1 - b1)(g - m),
// v <- b2 v + (1 - b2) g^2, p <- p - (lr / bc1) m / (sqrt(v) / sqrt(bc2) + eps)
// with bc1 = 1 - b1^t, bc2 = 1 - b2^t (passed in as step_*, bc2_sqrt).
__device__ __forceinline__ void adam1(float& p, float g, float& m, float& v, float step, float b1, float b2,
                                      float bc2_sqrt, float eps)
{
    m = m + (1.0f - b1) * (g - m);
    v = b2 * v + (1.0f - b2) * g * g;
    p = p - step * (m / (sqrtf(v) / bc2_sqrt + eps));
}

__global__ void k_adam(float4* __restrict__ p, const float4* __restrict__ g, float4* __restrict__ m,
                       float4* __restrict__ v, int64_t n4, float step_value, float step_deriv, float b1, float b2,
                       float bc2_sqrt, float eps)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n4) return;
    float4 pp = p[i], mm = m[i], vv = v[i];
    const float4 gg = g[i];
    adam1(pp.x, gg.x, mm.x, vv.x, step_value, b1, b2, bc2_sqrt, eps);
    adam1(pp.y, gg.y, mm.y, vv.y, step_deriv, b1, b2, bc2_sqrt, eps);
    adam1(pp.z, gg.z, mm.z, vv.z, step_deriv, b1, b2, bc2_sqrt, eps);
    adam1(pp.w, gg.w, mm.w, vv.w, step_deriv, b1, b2, bc2_sqrt, eps);
    p[i] = pp;
    m[i] = mm;
    v[i] = vv;
}

int launch_fit_loss_grad(const float* out, const float* dirs, const float* tr, const float* tn, int64_t Q,
                         float w_value, float* grad, hipStream_t stream)
{
    if (Q == 0) return SHM_OK;
    const int64_t blocks = (Q + 255) / 256;
    if (blocks > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "fit_loss_grad: too many queries");
    hipLaunchKernelGGL(k_fit_loss_grad, dim3((unsigned)blocks), dim3(256), 0, stream,
                       reinterpret_cast<const float4*>(out), dirs, tr, tn, Q, w_value, (float)(1.0 / (double)Q),
                       reinterpret_cast<float4*>(grad));
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

int launch_fit_forward_loss_grad(const float* lut, int N, const float* dirs, const float* tr, const float* tn,
                                 int64_t Q, float w_value, float* grad, hipStream_t stream)
{
    if (Q == 0) return SHM_OK;
    const int64_t blocks = (Q + 255) / 256;
    if (blocks > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "fit_forward_loss_grad: too many queries");
    hipLaunchKernelGGL(k_fit_forward_loss_grad, dim3((unsigned)blocks), dim3(256), 0, stream, lut, N, dirs, tr, tn, Q,
                       w_value, (float)(1.0 / (double)Q), reinterpret_cast<float4*>(grad));
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

int launch_adam(float* p, const float* g, float* m, float* v, int64_t n4, int64_t step, float lr_value,
                float lr_deriv, float b1, float b2, float eps, hipStream_t stream)
{
    if (n4 == 0) return SHM_OK;
    const int64_t blocks = (n4 + 255) / 256;
    if (blocks > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "adam: too many parameters");
    // bias corrections in double, as the reference optimiser forms them
    const double bc1 = 1.0 - std::pow((double)b1, (double)step);
    const double bc2 = 1.0 - std::pow((double)b2, (double)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, stream, reinterpret_cast<float4*>(p),
                       reinterpret_cast<const float4*>(g), reinterpret_cast<float4*>(m),
                       reinterpret_cast<float4*>(v), n4, (float)(lr_value / bc1), (float)(lr_deriv / bc1), b1, b2,
                       (float)std::sqrt(bc2), eps);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

}  // namespace shm
