// Radial depth of a triangle mesh (Sec. 4.9, mesh LOD impostors):
// R(w) = max{t >= 0 : c + t w on the mesh surface} for a set of directions
// (the sample grid of the finite-difference bake), computed by casting one
// ray per direction from the centre c against every triangle.
//
// Work decomposition: a workgroup owns RAYS rays (two per lane) and one
// chunk of triangles; the chunk streams through LDS in tiles of TRI_TILE triangles,
// and every lane tests its ray against the whole tile (all lanes read the
// same triangle: an LDS broadcast).
// Splitting the triangles over a second grid dimension fills the chip even
// for a few thousand rays; the chunks combine with an integer atomicMax on
// the bits of t >= 0 (order-preserving for non-negative floats), so the
// result does not depend on the order in which chunks finish.
//
// Intersection: c + t w = v0 + a e1 + b e2, solved with the scalar triple
// products of the ray-triangle (Moeller-Trumbore) form.  Every ray starts
// at c, so with s = c - v0 the products that do not involve w are the
// triangle's own: staged once per triangle are m = e2 x e1, u = e2 x s,
// q = s x e1 and t_num = e2 . q, and a ray then needs three dot products:
// det = w . m, a = (w . u)/det, b = (w . q)/det, t = t_num/det.  A hit needs
// a >= -eps, b >= -eps, a + b <= 1 + eps and t >= 0, with eps a few ulps
// so that rays through shared edges and vertices are not lost between the
// triangles around them.  det = 0 (a ray in the triangle's plane, or a
// degenerate triangle) gives an infinite reciprocal and a NaN or infinite
// a or a + b, which fails those tests.
#include "shm_device.hpp"
#include "shm_internal.hpp"

namespace shm {

constexpr int MESH_THREADS = 256;    // lanes per workgroup
constexpr int MESH_RPL = 2;          // rays per lane: each triangle read from LDS serves two tests
constexpr int MESH_RAYS = MESH_THREADS * MESH_RPL;  // rays per workgroup
constexpr int MESH_TILE = 256;       // triangles staged in LDS at a time
constexpr int MESH_CHUNK = 2048;     // triangles per workgroup

__global__ __launch_bounds__(MESH_THREADS) void k_mesh_depth(const float* __restrict__ verts, int64_t V,
                                                             const int32_t* __restrict__ tris, int64_t T, float cx,
                                                             float cy, float cz, const float* __restrict__ dirs,
                                                             int64_t P, unsigned int* __restrict__ best_bits)
{
    __shared__ float4 tri[MESH_TILE][3];  // (m, t_num), (u, -), (q, -): three 16-byte broadcast reads
    const int64_t f_begin = (int64_t)blockIdx.y * MESH_CHUNK;
    const int64_t f_end = min(f_begin + MESH_CHUNK, T);
    // ray j of this lane: blockIdx.x * MESH_RAYS + j * MESH_THREADS + threadIdx.x;
    // a ray past the end or with a zero or non-finite direction is dead:
    // w = 0 makes det = 0, which no test passes
    float wx[MESH_RPL], wy[MESH_RPL], wz[MESH_RPL], best[MESH_RPL];
    bool live[MESH_RPL];
#pragma unroll
    for (int j = 0; j < MESH_RPL; ++j) {
        const int64_t r = (int64_t)blockIdx.x * MESH_RAYS + j * MESH_THREADS + threadIdx.x;
        wx[j] = wy[j] = wz[j] = best[j] = 0.0f;
        live[j] = false;
        if (r < P) {
            const float x = dirs[3 * r], y = dirs[3 * r + 1], z = dirs[3 * r + 2];
            const float n2 = x * x + y * y + z * z;
            live[j] = n2 > 0.0f && isfinite(n2);
            if (live[j]) {
                const float in = rsqrtf(n2);
                wx[j] = x * in;
                wy[j] = y * in;
                wz[j] = z * in;
            }
        }
    }
    const float eps = 4.0f * 1.1920929e-7f;
    for (int64_t f0 = f_begin; f0 < f_end; f0 += MESH_TILE) {
        __syncthreads();  // the previous tile is no longer read
        const int64_t f = f0 + threadIdx.x;
        if (f < f_end) {
            const int64_t i0 = tris[3 * f], i1 = tris[3 * f + 1], i2 = tris[3 * f + 2];
            float4* d = tri[threadIdx.x];
            if (i0 >= 0 && i0 < V && i1 >= 0 && i1 < V && i2 >= 0 && i2 < V) {
                const float ax = verts[3 * i0], ay = verts[3 * i0 + 1], az = verts[3 * i0 + 2];
                const float sx = cx - ax, sy = cy - ay, sz = cz - az;
                const float e1x = verts[3 * i1] - ax, e1y = verts[3 * i1 + 1] - ay, e1z = verts[3 * i1 + 2] - az;
                const float e2x = verts[3 * i2] - ax, e2y = verts[3 * i2 + 1] - ay, e2z = verts[3 * i2 + 2] - az;
                const float qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
                d[0] = make_float4(e2y * e1z - e2z * e1y, e2z * e1x - e2x * e1z, e2x * e1y - e2y * e1x,
                                   e2x * qx + e2y * qy + e2z * qz);
                d[1] = make_float4(e2y * sz - e2z * sy, e2z * sx - e2x * sz, e2x * sy - e2y * sx, 0.0f);
                d[2] = make_float4(qx, qy, qz, 0.0f);
            } else {  // invalid index: a degenerate triangle (det = 0) no ray meets
                d[0] = d[1] = d[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
        __syncthreads();
        const int n = (int)min((int64_t)MESH_TILE, f_end - f0);
        for (int k = 0; k < n; ++k) {
            const float4 m = tri[k][0], u = tri[k][1], q = tri[k][2];
#pragma unroll
            for (int j = 0; j < MESH_RPL; ++j) {
                const float det = wx[j] * m.x + wy[j] * m.y + wz[j] * m.z;
                const float inv = __builtin_amdgcn_rcpf(det);  // ~1 ulp: t to a few ulps
                const float a = (wx[j] * u.x + wy[j] * u.y + wz[j] * u.z) * inv;
                const float b = (wx[j] * q.x + wy[j] * q.y + wz[j] * q.z) * inv;
                const float t = m.w * inv;
                if (a >= -eps && b >= -eps && a + b <= 1.0f + eps && t > best[j]) best[j] = t;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < MESH_RPL; ++j) {
        const int64_t r = (int64_t)blockIdx.x * MESH_RAYS + j * MESH_THREADS + threadIdx.x;
        if (live[j] && best[j] > 0.0f) atomicMax(best_bits + r, __float_as_uint(best[j]));
    }
}

__global__ void k_zero_u32(unsigned int* __restrict__ a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0u;
}

int launch_mesh_depth(const float* verts, int64_t V, const int32_t* tris, int64_t T, const float* center,
                      const float* dirs, int64_t P, float* depth, hipStream_t stream)
{
    if (P == 0) return SHM_OK;
    unsigned int* bits = reinterpret_cast<unsigned int*>(depth);  // t >= 0: max over the bits is max over t
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, stream, bits, P);
    SHM_LAUNCH_CHECK();
    if (T == 0) return SHM_OK;
    const int64_t gx = (P + MESH_RAYS - 1) / MESH_RAYS, gy = (T + MESH_CHUNK - 1) / MESH_CHUNK;
    if (gx > 0x7fffffff || gy > 65535) return fail(SHM_ERR_UNSUPPORTED, "mesh_depth: too many rays or triangles");
    hipLaunchKernelGGL(k_mesh_depth, dim3((unsigned)gx, (unsigned)gy), dim3(MESH_THREADS), 0, stream, verts, V, tris, T,
                       center[0], center[1], center[2], dirs, P, bits);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

}  // namespace shm
