// Backward of the query (differentiation form) for FP32 TEXEL LUTs.
//
// The outputs (R, grad R) are linear in the 16 footprint scalars, so
// dL/dLUT is a scatter of per-query weights onto 4 texels.  To make it
// deterministic without floating-point atomics:
//   1. sort:   cell key per query, stable LSD radix sort (8-bit digits) of
//              (key, query index) -> permutation, cell segment starts, rank
//   2. query:  per query (original order) the direction gradient (second
//              chart derivatives + derivative of the chart map) and a compact
//              record (s, t, gR, N lambda_u, N lambda_v) stored at its rank
//   3. cells:  per cell, the sum over its sorted query segment of the 16
//              weights (4 corners x 4 channels), in segment order
//   4. texels: per texel, the corner sums of its <= 4 adjacent cells in a
//              fixed order
// The sort depends only on the directions and is reused while they stay
// fixed.  Integer atomics appear only in the per-block digit histograms.
#include "shm_device.hpp"
#include "shm_internal.hpp"

namespace shm {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;                       // elements per thread per tile
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;     // 4096 elements per block
constexpr uint32_t KEY_INVALID = 0xffffffffu;
constexpr int SC_THREADS = 256, SC_ITEMS = 16, SC_TILE = SC_THREADS * SC_ITEMS;  // scan tiles

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct BwdLayout {
    size_t keys0, vals0, keys1, vals1, rank, cstart, hist, tsum, rec4, rec1, csum, total;
    int64_t Q, n_cells, nb;
    int passes;
};

static BwdLayout bwd_layout(int N, int64_t n_obj, int64_t q_per_obj)
{
    BwdLayout W;
    W.Q = n_obj * q_per_obj;
    W.n_cells = n_obj * 6ll * (N + 1) * (N + 1);
    W.nb = (W.Q + RS_TILE - 1) / RS_TILE;
    int bits = 1;
    while (((int64_t)1 << bits) <= W.n_cells) ++bits;  // keys 0..n_cells (n_cells = invalid bucket)
    W.passes = (bits + 7) / 8;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
    W.keys0 = take(W.Q * 4);
    W.vals0 = take(W.Q * 4);
    W.keys1 = take(W.Q * 4);
    W.vals1 = take(W.Q * 4);
    W.rank = take(W.Q * 4);
    W.cstart = take((W.n_cells + 1) * 4);
    W.hist = take((size_t)256 * W.nb * 4);
    W.tsum = take(((size_t)256 * W.nb + SC_TILE - 1) / SC_TILE * 4);
    W.rec4 = take(W.Q * 16);
    W.rec1 = take(W.Q * 4);
    W.csum = take(W.n_cells * 64);
    W.total = o;
    return W;
}

size_t backward_workspace_bytes(int N, int64_t n_obj, int64_t q_per_obj)
{
    return bwd_layout(N, n_obj, q_per_obj).total;
}

// ---------------------------------------------------------------------------
// cell keys
// ---------------------------------------------------------------------------
__global__ void k_cell_keys(int N, int64_t Q, int64_t q_per_obj, const float* __restrict__ dirs,
                            uint32_t invalid_key, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    const Loc L = locate(dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2], N);
    const int64_t C = N + 1;
    const int64_t obj = q / q_per_obj;
    keys[q] = L.face < 0 ? invalid_key : (uint32_t)(((obj * 6 + L.face) * C + L.j0) * C + L.i0);
    if (vals) vals[q] = (uint32_t)q;
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, one 8-bit digit per pass
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t Q, int shift,
                                                           int64_t nb, uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * RS_TILE;
    for (int i = threadIdx.x; i < RS_TILE; i += RS_THREADS) {
        const int64_t e = t0 + i;
        if (e < Q) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of n uint32: per-block scans of 4096 elements (256 lanes x
// 16), a one-workgroup scan of the block totals, then the block offsets

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total)
{
    // Hillis-Steele over the 256 lanes of the workgroup
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < SC_THREADS; off <<= 1) {
        const uint32_t a = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    const uint32_t incl = sh[t];
    *total = sh[SC_THREADS - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(SC_THREADS) void k_scan_tiles(uint32_t* __restrict__ a, int64_t n,
                                                           uint32_t* __restrict__ tile_sums)
{
    __shared__ uint32_t sh[SC_THREADS];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
    uint32_t v[SC_ITEMS], sum = 0;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        v[i] = (base + i < n) ? a[base + i] : 0u;
        sum += v[i];
    }
    uint32_t total;
    uint32_t run = block_excl_scan(sum, sh, &total);
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        if (base + i < n) a[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// one workgroup: exclusive scan of the tile sums (any count, chunks of 256)
__global__ __launch_bounds__(SC_THREADS) void k_scan_sums(uint32_t* __restrict__ s, int64_t n)
{
    __shared__ uint32_t sh[SC_THREADS];
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < n; c0 += SC_THREADS) {
        const int64_t i = c0 + threadIdx.x;
        const uint32_t v = i < n ? s[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan(v, sh, &total);
        if (i < n) s[i] = carry + ex;
        carry += total;
    }
}

__global__ __launch_bounds__(SC_THREADS) void k_scan_add(uint32_t* __restrict__ a, int64_t n,
                                                         const uint32_t* __restrict__ tile_sums)
{
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
    const uint32_t add = tile_sums[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i)
        if (base + i < n) a[base + i] += add;
}

__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                              const uint32_t* __restrict__ vin, int64_t Q, int shift,
                                                              int64_t nb, const uint32_t* __restrict__ offs,
                                                              uint32_t* __restrict__ kout, uint32_t* __restrict__ vout)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t cnt[4][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    run[tid] = offs[(int64_t)tid * nb + blockIdx.x];
    const int64_t t0 = (int64_t)blockIdx.x * RS_TILE;
    const unsigned long long lt = (1ull << lane) - 1ull;
    for (int c = 0; c < RS_ITEMS; ++c) {
        for (int k = 0; k < 4; ++k) cnt[k][tid] = 0;
        __syncthreads();
        const int64_t e = t0 + (int64_t)c * RS_THREADS + tid;
        const bool valid = e < Q;
        const uint32_t key = valid ? kin[e] : 0u;
        const uint32_t val = valid ? vin[e] : 0u;
        const uint32_t d = (key >> shift) & 255u;
        // lanes of this wave holding the same digit (valid lanes only)
        unsigned long long same = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            const unsigned long long bb = __ballot((d >> bit) & 1u);
            same &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const uint32_t r_in_wave = (uint32_t)__popcll(same & lt);
        if (valid && r_in_wave == 0) cnt[w][d] = (uint32_t)__popcll(same);
        __syncthreads();
        // prefix over waves for digit tid
        const uint32_t c0 = cnt[0][tid], c1 = cnt[1][tid], c2 = cnt[2][tid], c3 = cnt[3][tid];
        __syncthreads();
        cnt[0][tid] = 0;
        cnt[1][tid] = c0;
        cnt[2][tid] = c0 + c1;
        cnt[3][tid] = c0 + c1 + c2;
        __syncthreads();
        if (valid) {
            const uint32_t pos = run[d] + cnt[w][d] + r_in_wave;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        run[tid] += c0 + c1 + c2 + c3;
        __syncthreads();
    }
}

// cell_start[c] = first sorted position with key >= c, c = 0..n_cells
__global__ void k_cell_start(const uint32_t* __restrict__ sk, int64_t Q, int64_t n_cells, uint32_t* __restrict__ cs)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > n_cells) return;
    int64_t lo = 0, hi = Q;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)sk[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    cs[c] = (uint32_t)lo;
}

__global__ void k_inverse_perm(const uint32_t* __restrict__ perm, int64_t Q, uint32_t* __restrict__ rank)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < Q) rank[perm[k]] = (uint32_t)k;
}

int launch_backward_sort(int N, int64_t n_obj, const float* dirs, int64_t q_per_obj, void* ws, hipStream_t stream)
{
    const BwdLayout W = bwd_layout(N, n_obj, q_per_obj);
    if (W.Q == 0) return SHM_OK;
    char* base = reinterpret_cast<char*>(ws);
    uint32_t* k0 = reinterpret_cast<uint32_t*>(base + W.keys0);
    uint32_t* v0 = reinterpret_cast<uint32_t*>(base + W.vals0);
    uint32_t* k1 = reinterpret_cast<uint32_t*>(base + W.keys1);
    uint32_t* v1 = reinterpret_cast<uint32_t*>(base + W.vals1);
    uint32_t* hist = reinterpret_cast<uint32_t*>(base + W.hist);
    uint32_t* tsum = reinterpret_cast<uint32_t*>(base + W.tsum);
    const int64_t n_hist = (int64_t)256 * W.nb;
    const int64_t n_tiles = (n_hist + SC_TILE - 1) / SC_TILE;
    const unsigned gq = (unsigned)((W.Q + 255) / 256);
    hipLaunchKernelGGL(k_cell_keys, dim3(gq), dim3(256), 0, stream, N, W.Q, q_per_obj, dirs, (uint32_t)W.n_cells, k0, v0);
    SHM_LAUNCH_CHECK();
    for (int p = 0; p < W.passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)W.nb), dim3(RS_THREADS), 0, stream, k0, W.Q, shift, W.nb, hist);
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)n_tiles), dim3(SC_THREADS), 0, stream, hist, n_hist, tsum);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SC_THREADS), 0, stream, tsum, n_tiles);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)n_tiles), dim3(SC_THREADS), 0, stream, hist, n_hist, tsum);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)W.nb), dim3(RS_THREADS), 0, stream, k0, v0, W.Q, shift, W.nb,
                           hist, k1, v1);
        SHM_LAUNCH_CHECK();
        uint32_t* t = k0; k0 = k1; k1 = t;
        t = v0; v0 = v1; v1 = t;
    }
    // sorted keys in k0, permutation in v0 (buffer 0 or 1 depending on parity)
    uint32_t* cs = reinterpret_cast<uint32_t*>(base + W.cstart);
    uint32_t* rank = reinterpret_cast<uint32_t*>(base + W.rank);
    hipLaunchKernelGGL(k_cell_start, dim3((unsigned)((W.n_cells + 1 + 255) / 256)), dim3(256), 0, stream, k0, W.Q,
                       W.n_cells, cs);
    hipLaunchKernelGGL(k_inverse_perm, dim3(gq), dim3(256), 0, stream, v0, W.Q, rank);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

int launch_cell_keys(int N, int64_t n_obj, const float* dirs, int64_t q_per_obj, uint32_t* keys, hipStream_t stream)
{
    const int64_t Q = n_obj * q_per_obj;
    if (Q == 0) return SHM_OK;
    hipLaunchKernelGGL(k_cell_keys, dim3((unsigned)((Q + 255) / 256)), dim3(256), 0, stream, N, Q, q_per_obj, dirs,
                       KEY_INVALID, keys, (uint32_t*)nullptr);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

// ---------------------------------------------------------------------------
// per-query pass: direction gradient and the record at the query's rank
// ---------------------------------------------------------------------------
__global__ void k_bwd_query(const float* __restrict__ lut, int N, int64_t lut_elems, int64_t Q, int64_t q_per_obj,
                            const float* __restrict__ dirs, const float* __restrict__ gout,
                            const uint32_t* __restrict__ rank, float4* __restrict__ rec4, float* __restrict__ rec1,
                            float* __restrict__ grad_dirs)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    const float x = dirs[3 * q], y = dirs[3 * q + 1], z = dirs[3 * q + 2];
    const Loc L = locate(x, y, z, N);
    const uint32_t pos = rank[q];
    if (L.face < 0) {
        rec4[pos] = make_float4(0.f, 0.f, 0.f, 0.f);
        rec1[pos] = 0.f;
        if (grad_dirs) {
            const float nan = __builtin_nanf("");
            grad_dirs[3 * q] = nan;
            grad_dirs[3 * q + 1] = nan;
            grad_dirs[3 * q + 2] = nan;
        }
        return;
    }
    const float4 g = reinterpret_cast<const float4*>(gout)[q];
    const float gR = g.x;
    float3 M, S, T;
    frame_of(L.face, M, S, T);
    const float a = L.a, b = L.b;
    const float3 Sa = make_float3(S.x - a * M.x, S.y - a * M.y, S.z - a * M.z);
    const float3 Tb = make_float3(T.x - b * M.x, T.y - b * M.y, T.z - b * M.z);
    const float gS = g.y * Sa.x + g.z * Sa.y + g.w * Sa.z;
    const float gT = g.y * Tb.x + g.z * Tb.y + g.w * Tb.z;
    const float rho = sqrtf(1.0f + a * a + b * b);
    const float k = 0.5f * rho;
    const float Nf = (float)N;
    const float lu = k * gS, lv = k * gT;  // dL/dr_u, dL/dr_v
    rec4[pos] = make_float4(L.s, L.t, gR, Nf * lu);
    rec1[pos] = Nf * lv;
    if (grad_dirs) {
        const int64_t obj = q / q_per_obj;
        const Foot F = load_texel_f32(lut + obj * lut_elems, N, L);
        const Patch2 P = hermite2(F, L.s, L.t);
        const float gM = g.y * M.x + g.z * M.y + g.w * M.z;
        const float ru = Nf * P.rs, rv = Nf * P.rt;
        const float hN2 = 0.5f * Nf * Nf;
        const float common = (ru * gS + rv * gT) / (2.0f * rho);
        const float dLda = 0.5f * Nf * gR * P.rs + a * common + k * (hN2 * P.rss * gS - ru * gM + hN2 * P.rst * gT);
        const float dLdb = 0.5f * Nf * gR * P.rt + b * common + k * (hN2 * P.rst * gS + hN2 * P.rtt * gT - rv * gM);
        const float ma = x * M.x + y * M.y + z * M.z;
        const float im = 1.0f / ma;
        grad_dirs[3 * q] = (dLda * Sa.x + dLdb * Tb.x) * im;
        grad_dirs[3 * q + 1] = (dLda * Sa.y + dLdb * Tb.y) * im;
        grad_dirs[3 * q + 2] = (dLda * Sa.z + dLdb * Tb.z) * im;
    }
}

// ---------------------------------------------------------------------------
// cell pass: csum[c][corner] (float4 over channels) = sum over the queries of
// cell c, in sorted order, of that corner's 4 channel weights
// ---------------------------------------------------------------------------
__global__ void k_bwd_cells(int64_t n_cells, const uint32_t* __restrict__ cs, const float4* __restrict__ rec4,
                            const float* __restrict__ rec1, float4* __restrict__ csum)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const uint32_t kb = cs[c], ke = cs[c + 1];
    float4 a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (uint32_t kk = kb; kk < ke; ++kk) {
        const float4 r = rec4[kk];
        const float nlv = rec1[kk];
        const Basis1 S = basis1(r.x), T = basis1(r.y);
        const float gR = r.z, nlu = r.w;
#pragma unroll
        for (int corner = 0; corner < 4; ++corner) {
            const bool ci = corner & 1, cj = corner >> 1;
            const float Hi = ci ? S.h1 : 1.0f - S.h1, Hdi = ci ? S.h1d : S.h0d;
            const float dHi = ci ? S.d1 : -S.d1, dHdi = ci ? S.d1d : S.d0d;
            const float Hj = cj ? T.h1 : 1.0f - T.h1, Hdj = cj ? T.h1d : T.h0d;
            const float dHj = cj ? T.d1 : -T.d1, dHdj = cj ? T.d1d : T.d0d;
            a[corner].x += gR * Hi * Hj + nlu * dHi * Hj + nlv * Hi * dHj;
            a[corner].y += gR * Hdi * Hj + nlu * dHdi * Hj + nlv * Hdi * dHj;
            a[corner].z += gR * Hi * Hdj + nlu * dHi * Hdj + nlv * Hi * dHdj;
            a[corner].w += gR * Hdi * Hdj + nlu * dHdi * Hdj + nlv * Hdi * dHdj;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) csum[c * 4 + k] = a[k];
}

// ---------------------------------------------------------------------------
// texel pass: grad_lut[texel] = sum over its adjacent cells (fixed order) of
// the cell sum of the corner this texel is
// ---------------------------------------------------------------------------
__global__ void k_bwd_texels(int N, int64_t n_tex, const float4* __restrict__ csum, float4* __restrict__ grad_lut)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_tex) return;
    const int P = N + 2, C = N + 1;
    const int64_t per = 6ll * P * P;
    const int64_t obj = i / per;
    const int rem = (int)(i - obj * per);
    const int face = rem / (P * P), r2 = rem - face * P * P;
    const int q = r2 / P, p = r2 - q * P;
    const int64_t cell_base = (obj * 6 + face) * (int64_t)C * C;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int dj = 1; dj >= 0; --dj) {
        const int j0 = q - dj;
        if (j0 < 0 || j0 > N) continue;
        for (int di = 1; di >= 0; --di) {
            const int i0 = p - di;
            if (i0 < 0 || i0 > N) continue;
            const float4 v = csum[(cell_base + (int64_t)j0 * C + i0) * 4 + (dj * 2 + di)];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
    }
    grad_lut[i] = acc;
}

int launch_backward(const float* lut, int N, int64_t n_obj, const float* dirs, int64_t q_per_obj, const float* gout,
                    float* grad_lut, float* grad_dirs, void* ws, hipStream_t stream)
{
    const BwdLayout W = bwd_layout(N, n_obj, q_per_obj);
    char* base = reinterpret_cast<char*>(ws);
    const uint32_t* cs = reinterpret_cast<const uint32_t*>(base + W.cstart);
    const uint32_t* rank = reinterpret_cast<const uint32_t*>(base + W.rank);
    float4* rec4 = reinterpret_cast<float4*>(base + W.rec4);
    float* rec1 = reinterpret_cast<float*>(base + W.rec1);
    if (W.Q > 0) {
        hipLaunchKernelGGL(k_bwd_query, dim3((unsigned)((W.Q + 255) / 256)), dim3(256), 0, stream, lut, N,
                           texel_elems(N), W.Q, q_per_obj, dirs, gout, rank, rec4, rec1, grad_dirs);
        SHM_LAUNCH_CHECK();
    }
    if (grad_lut) {
        float4* csum = reinterpret_cast<float4*>(base + W.csum);
        hipLaunchKernelGGL(k_bwd_cells, dim3((unsigned)((W.n_cells + 255) / 256)), dim3(256), 0, stream, W.n_cells, cs,
                           rec4, rec1, csum);
        const int64_t n_tex = n_obj * 6ll * (N + 2) * (N + 2);
        hipLaunchKernelGGL(k_bwd_texels, dim3((unsigned)((n_tex + 255) / 256)), dim3(256), 0, stream, N, n_tex, csum,
                           reinterpret_cast<float4*>(grad_lut));
        SHM_LAUNCH_CHECK();
    }
    return SHM_OK;
}

}  // namespace shm
