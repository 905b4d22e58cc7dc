// Radial depth of a triangle mesh (Sec. 4.9, mesh LOD impostors):
// R(w) = max{t >= 0 : c + t w on the mesh surface} for a set of directions
// (the sample grid of the finite-difference bake), computed by casting one
// ray per direction from the centre c against every triangle.
//
// Work decomposition: a workgroup owns RAYS rays and one chunk of
// triangles; the chunk streams through LDS in tiles of TRI_TILE triangles
// (each staged once as v0 - c, e1, e2), and every lane tests its ray against
// the whole tile (all lanes read the same triangle: an LDS broadcast).
// Splitting the triangles over a second grid dimension fills the chip even
// for a few thousand rays; the chunks combine with an integer atomicMax on
// the bits of t >= 0 (order-preserving for non-negative floats), so the
// result does not depend on the order in which chunks finish.
//
// Intersection: c + t w = v0 + a e1 + b e2, solved with the scalar triple
// products of the ray-triangle (Moeller-Trumbore) form; a hit needs
// a >= -eps, b >= -eps, a + b <= 1 + eps and t >= 0, with eps a few ulps
// so that rays through shared edges and vertices are not lost between the
// triangles around them.
#include "shm_device.hpp"
#include "shm_internal.hpp"

namespace shm {

constexpr int MESH_RAYS = 256;       // rays (lanes) per workgroup
constexpr int MESH_TILE = 256;       // triangles staged in LDS at a time
constexpr int MESH_CHUNK = 4096;     // triangles per workgroup

__global__ __launch_bounds__(MESH_RAYS) void k_mesh_depth(const float* __restrict__ verts, int64_t V,
                                                          const int32_t* __restrict__ tris, int64_t T, float cx,
                                                          float cy, float cz, const float* __restrict__ dirs,
                                                          int64_t P, unsigned int* __restrict__ best_bits)
{
    __shared__ float4 tri[MESH_TILE][3];  // v0 - c, e1, e2 (w unused): three 16-byte broadcast reads
    const int64_t r = (int64_t)blockIdx.x * MESH_RAYS + threadIdx.x;
    const int64_t f_begin = (int64_t)blockIdx.y * MESH_CHUNK;
    const int64_t f_end = min(f_begin + MESH_CHUNK, T);
    float wx = 0.f, wy = 0.f, wz = 0.f;
    bool live = false;
    if (r < P) {
        wx = dirs[3 * r];
        wy = dirs[3 * r + 1];
        wz = dirs[3 * r + 2];
        const float n2 = wx * wx + wy * wy + wz * wz;
        live = n2 > 0.0f && isfinite(n2);
        if (live) {
            const float in = rsqrtf(n2);
            wx *= in;
            wy *= in;
            wz *= in;
        }
    }
    const float eps = 4.0f * 1.1920929e-7f;
    float best = 0.0f;
    for (int64_t f0 = f_begin; f0 < f_end; f0 += MESH_TILE) {
        __syncthreads();  // the previous tile is no longer read
        const int64_t f = f0 + threadIdx.x;
        if (f < f_end) {
            const int64_t i0 = tris[3 * f], i1 = tris[3 * f + 1], i2 = tris[3 * f + 2];
            float4* d = tri[threadIdx.x];
            if (i0 >= 0 && i0 < V && i1 >= 0 && i1 < V && i2 >= 0 && i2 < V) {
                const float ax = verts[3 * i0], ay = verts[3 * i0 + 1], az = verts[3 * i0 + 2];
                d[0] = make_float4(ax - cx, ay - cy, az - cz, 0.0f);
                d[1] = make_float4(verts[3 * i1] - ax, verts[3 * i1 + 1] - ay, verts[3 * i1 + 2] - az, 0.0f);
                d[2] = make_float4(verts[3 * i2] - ax, verts[3 * i2 + 1] - ay, verts[3 * i2 + 2] - az, 0.0f);
            } else {  // invalid index: a degenerate triangle (det = 0) no ray meets
                d[0] = d[1] = d[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
        __syncthreads();
        const int n = (int)min((int64_t)MESH_TILE, f_end - f0);
        if (live) {
            for (int k = 0; k < n; ++k) {
                const float4 o = tri[k][0], e1 = tri[k][1], e2 = tri[k][2];
                const float e1x = e1.x, e1y = e1.y, e1z = e1.z, e2x = e2.x, e2y = e2.y, e2z = e2.z;
                // p = w x e2, det = e1 . p
                const float px = wy * e2z - wz * e2y, py = wz * e2x - wx * e2z, pz = wx * e2y - wy * e2x;
                const float det = e1x * px + e1y * py + e1z * pz;
                if (det == 0.0f) continue;
                const float inv = __builtin_amdgcn_rcpf(det);  // ~1 ulp: t to a few ulps
                // s = c - v0 = -(v0 - c)
                const float sx = -o.x, sy = -o.y, sz = -o.z;
                const float a = (sx * px + sy * py + sz * pz) * inv;
                const float qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
                const float b = (wx * qx + wy * qy + wz * qz) * inv;
                const float t = (e2x * qx + e2y * qy + e2z * qz) * inv;
                if (a >= -eps && b >= -eps && a + b <= 1.0f + eps && t > best) best = t;
            }
        }
    }
    if (live && best > 0.0f) atomicMax(best_bits + r, __float_as_uint(best));
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
    hipLaunchKernelGGL(k_mesh_depth, dim3((unsigned)gx, (unsigned)gy), dim3(MESH_RAYS), 0, stream, verts, V, tris, T,
                       center[0], center[1], center[2], dirs, P, bits);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

}  // namespace shm
