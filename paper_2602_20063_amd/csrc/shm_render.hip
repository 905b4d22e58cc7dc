// Query of the rendered radius (Sec. 3.1): R = s r for a nonnegative
// function, R = s |r| for a signed one, with the gradient and normal of
// Sec. 3.4 (Eq. 10 with grad R = s sign(r) grad r) and the sign of r for
// shading.  Same gather and Hermite evaluation as the plain query; one lane
// per query, objects of one face size back to back.
#include "shm_device.hpp"
#include "shm_internal.hpp"

namespace shm {

template <bool FP16, bool CELL>
__global__ __launch_bounds__(256) void k_query_scaled(const void* __restrict__ lut, int N, int64_t lut_elems,
                                                      int64_t q_per_obj, int tiles_per_obj,
                                                      const float* __restrict__ dirs, float scale, int is_signed,
                                                      float* __restrict__ out, float* __restrict__ nrm,
                                                      int8_t* __restrict__ sign)
{
    const int b = (int)blockIdx.x;
    const int obj = b / tiles_per_obj;
    const int64_t ql = (int64_t)(b - obj * tiles_per_obj) * 256 + threadIdx.x;
    if (ql >= q_per_obj) return;
    const int64_t q = (int64_t)obj * q_per_obj + ql;
    const char* base = reinterpret_cast<const char*>(lut) + (size_t)obj * (size_t)lut_elems * (FP16 ? 2 : 4);
    const float x = dirs[3 * q], y = dirs[3 * q + 1], z = dirs[3 * q + 2];
    int sg;
    const float4 r = rendered(query_one<FP16, CELL>(base, N, x, y, z), scale, is_signed != 0, &sg);
    reinterpret_cast<float4*>(out)[q] = r;
    if (nrm) {
        const float3 n = normal_of(r.x, x, y, z, make_float3(r.y, r.z, r.w));
        nrm[3 * q] = n.x;
        nrm[3 * q + 1] = n.y;
        nrm[3 * q + 2] = n.z;
    }
    if (sign) sign[q] = (int8_t)sg;
}

int launch_query_scaled(const void* lut, int dtype, int layout, int N, int64_t n_obj, const float* dirs,
                        int64_t q_per_obj, float scale, int flags, float* out, float* normal, int8_t* sign,
                        hipStream_t stream)
{
    if (n_obj == 0 || q_per_obj == 0) return SHM_OK;
    const int64_t tiles = (q_per_obj + 255) / 256;
    if (tiles * n_obj > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "query_scaled: too many tiles for one launch");
    const dim3 grid((unsigned)(tiles * n_obj)), block(256);
    const int64_t le = layout == SHM_LAYOUT_CELL ? cell_elems(N) : texel_elems(N);
    const int sgn = (flags & SHM_SIGNED) ? 1 : 0;
    const int tpo = (int)tiles;
    if (dtype == SHM_F16) {
        if (layout == SHM_LAYOUT_CELL)
            hipLaunchKernelGGL((k_query_scaled<true, true>), grid, block, 0, stream, lut, N, le, q_per_obj, tpo, dirs, scale, sgn, out, normal, sign);
        else
            hipLaunchKernelGGL((k_query_scaled<true, false>), grid, block, 0, stream, lut, N, le, q_per_obj, tpo, dirs, scale, sgn, out, normal, sign);
    } else {
        if (layout == SHM_LAYOUT_CELL)
            hipLaunchKernelGGL((k_query_scaled<false, true>), grid, block, 0, stream, lut, N, le, q_per_obj, tpo, dirs, scale, sgn, out, normal, sign);
        else
            hipLaunchKernelGGL((k_query_scaled<false, false>), grid, block, 0, stream, lut, N, le, q_per_obj, tpo, dirs, scale, sgn, out, normal, sign);
    }
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

}  // namespace shm
