// Mip chain of a Spherical Hermite Map (Sec. 4.7, Table lod).
//
// Level k+1 (face size N/2) from level k (face size N, FP32 TEXEL):
//   consistent: the value field is box-filtered -- each coarse sample is the
//     mean of the level-k map at the four fine texel-centre directions the
//     coarse texel covers, taken as full queries so that points beyond the
//     face read the neighbouring face -- on the coarse padded grid plus a
//     margin ring; the derivative channels are then recomputed by central
//     differences (the general-mode bake).  This keeps the stored channels
//     the scaled derivatives of the filtered field (Eq. 2).
//   naive: as consistent, but every interior coarse texel holds the plain
//     average of the four fine texels' stored channels, as a box-filtering
//     mip generator would; the scaled derivative channels then no longer
//     describe the filtered field.
#include "shm_device.hpp"
#include "shm_internal.hpp"

namespace shm {

int launch_bake_fd(const float* samples, int N, int64_t n_obj, int out_dtype, void* lut, hipStream_t stream);

__global__ void k_mip_samples(const float* __restrict__ lut, int N, float* __restrict__ samples)
{
    const int Nc = N / 2, Pm = Nc + 4;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 6 * Pm * Pm) return;
    const int face = i / (Pm * Pm), rem = i - face * Pm * Pm;
    const int q = rem / Pm, p = rem - q * Pm;
    float3 M, S, T;
    frame_of(face, M, S, T);
    const float uc = ((float)p - 1.5f) / (float)Nc, vc = ((float)q - 1.5f) / (float)Nc;
    const float half = 0.5f / (float)N;
    float acc = 0.0f;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const float A = 2.0f * (uc + (a ? half : -half)) - 1.0f;
            const float B = 2.0f * (vc + (b ? half : -half)) - 1.0f;
            const float x = M.x + A * S.x + B * T.x, y = M.y + A * S.y + B * T.y, z = M.z + A * S.z + B * T.z;
            acc += query_one<false, false>(lut, N, x, y, z).x;
        }
    samples[i] = 0.25f * acc;
}

__global__ void k_mip_naive_interior(const float4* __restrict__ fine, int N, float4* __restrict__ coarse)
{
    const int Nc = N / 2, P = N + 2, Pc = Nc + 2;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 6 * Nc * Nc) return;
    const int face = i / (Nc * Nc), rem = i - face * Nc * Nc;
    const int q = rem / Nc + 1, p = rem % Nc + 1;  // interior coarse texel
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const float4 v = fine[((int64_t)face * P + (2 * q - 1 + b)) * P + (2 * p - 1 + a)];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
    coarse[((int64_t)face * Pc + q) * Pc + p] = make_float4(0.25f * acc.x, 0.25f * acc.y, 0.25f * acc.z, 0.25f * acc.w);
}

size_t mip_workspace_bytes(int N) { return (size_t)6 * (N / 2 + 4) * (N / 2 + 4) * sizeof(float); }

int launch_mip_level(const float* lut, int N, int mode, float* ws, float* out, hipStream_t stream)
{
    const int Nc = N / 2, Pm = Nc + 4;
    const int n = 6 * Pm * Pm;
    hipLaunchKernelGGL(k_mip_samples, dim3((n + 255) / 256), dim3(256), 0, stream, lut, N, ws);
    SHM_LAUNCH_CHECK();
    int rc = launch_bake_fd(ws, Nc, 1, SHM_F32, out, stream);
    if (rc) return rc;
    if (mode == 1) {
        const int m = 6 * Nc * Nc;
        hipLaunchKernelGGL(k_mip_naive_interior, dim3((m + 255) / 256), dim3(256), 0, stream,
                           reinterpret_cast<const float4*>(lut), N, reinterpret_cast<float4*>(out));
        SHM_LAUNCH_CHECK();
    }
    return SHM_OK;
}

}  // namespace shm
