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
// The whole step fused into one kernel is k_bwd_fused<FIT> beside the
// backward it extends.
#include "shm_device.hpp"
#include "shm_fit.hpp"
#include "shm_internal.hpp"

namespace shm {

__global__ void k_fit_loss_grad(const float4* __restrict__ out, const float* __restrict__ dirs,
                                const float* __restrict__ tr, const float* __restrict__ tn, int64_t Q, float w_value,
                                float inv_q, float4* __restrict__ grad)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    grad[q] = loss_grad_one(out[q], dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2], tr[q], tn[3 * q], tn[3 * q + 1],
                            tn[3 * q + 2], w_value, inv_q);
}

// The forward query of a FP32 TEXEL LUT fused with the loss gradient,
// without writing (R, grad R) out and reading it back; the fitting-step
// kernel runs the same arithmetic (fit_forward, loss_grad_one).
__global__ void k_fit_forward_loss_grad(const float* __restrict__ lut, int N, const float* __restrict__ dirs,
                                        const float* __restrict__ tr, const float* __restrict__ tn, int64_t Q,
                                        float w_value, float inv_q, float4* __restrict__ grad)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    const float x = dirs[3 * q], y = dirs[3 * q + 1], z = dirs[3 * q + 2];
    const Loc L = locate(x, y, z, N);
    const float nan = __builtin_nanf("");
    const float4 o = L.face < 0 ? make_float4(nan, nan, nan, nan) : fit_forward(lut, N, L);
    grad[q] = loss_grad_one(o, x, y, z, tr[q], tn[3 * q], tn[3 * q + 1], tn[3 * q + 2], w_value, inv_q);
}

__global__ void k_adam(float4* __restrict__ p, const float4* __restrict__ g, float4* __restrict__ m,
                       float4* __restrict__ v, int64_t n4, AdamConsts k)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n4) return;
    float4 pp = p[i], mm = m[i], vv = v[i];
    adam_texel(pp, g[i], mm, vv, k);
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
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, stream, reinterpret_cast<float4*>(p),
                       reinterpret_cast<const float4*>(g), reinterpret_cast<float4*>(m),
                       reinterpret_cast<float4*>(v), n4, adam_consts(step, lr_value, lr_deriv, b1, b2, eps));
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

}  // namespace shm
