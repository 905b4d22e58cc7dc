// Backward of the query (differentiation form) for FP32 TEXEL LUTs.
//
// The outputs (R, grad R) are linear in the 16 footprint scalars, so
// dL/dLUT is a scatter of per-query weights onto 4 texels.  To make it
// deterministic without floating-point atomics:
//   1. sort:   cell key per query, stable LSD radix sort (8-bit digits) of
//              (key, query index) -> permutation, cell segment starts
//   2. tiles:  one workgroup per 15 x 15 texel tile of a face; one lane per
//              cell of the tile (halo included) sums the 16 weights (4 corners
//              x 4 channels) of its sorted query segment in order; each texel
//              then adds its <= 4 cells' corner sums in a fixed order
//   3. dirs:   the direction gradient of each query (second chart derivatives
//              + derivative of the chart map), one lane per query in the
//              queries' own order: it involves no other query
// The sort depends only on the directions and is reused while they stay
// fixed.  Integer atomics appear only in the per-block digit histograms.
#include "shm_device.hpp"
#include "shm_fit.hpp"
#include "shm_internal.hpp"

// texels per LUT-gradient tile side (a compile-time tuning knob): BC * BC
// cells, one per lane of the tile's workgroup (256 lanes for 15, 1024 for 31)
#ifndef SHM_BWD_BT
#define SHM_BWD_BT 15
#endif

namespace shm {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;                       // elements per thread per tile
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;     // 4096 elements per block
constexpr uint32_t KEY_INVALID = 0xffffffffu;
constexpr int SC_THREADS = 256, SC_ITEMS = 16, SC_TILE = SC_THREADS * SC_ITEMS;  // scan tiles

static inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// dense-tile record of a sort: a uint32 count, the list of dense tiles
// (uint32 each, in no particular order) and one flag byte per tile
static inline size_t dense_bytes(int64_t n_tiles) { return 16 + (size_t)n_tiles * 5; }
struct DenseTiles {
    uint32_t* count;
    uint32_t* list;
    uint8_t* flag;
};
static inline DenseTiles dense_tiles(char* at, int64_t n_tiles)
{
    return DenseTiles{reinterpret_cast<uint32_t*>(at), reinterpret_cast<uint32_t*>(at + 16),
                      reinterpret_cast<uint8_t*>(at + 16 + (size_t)n_tiles * 4)};
}

struct BwdLayout {
    size_t keys0, vals0, keys1, vals1, cstart, hist, tsum, sdirs = 0, sgout = 0, dense = 0, geo = 0, total;
    int64_t Q, n_cells, nb, n_tiles = 0;
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
    W.cstart = take((W.n_cells + 1) * 4);
    W.hist = take((size_t)256 * W.nb * 4);
    W.tsum = take(((size_t)256 * W.nb + SC_TILE - 1) / SC_TILE * 4);
    const int64_t tpf = (N + 2 + SHM_BWD_BT - 1) / SHM_BWD_BT;
    W.n_tiles = n_obj * 6 * tpf * tpf;
    W.dense = take(dense_bytes(W.n_tiles));  // dense-tile count, list and flags
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
// the valid lanes of this wave whose digit equals this lane's digit d
__device__ __forceinline__ unsigned long long same_digit_lanes(uint32_t d, bool valid)
{
    unsigned long long same = __ballot(valid);
    // a round whose valid lanes share one digit (common where keys are
    // nearly in order) needs no per-bit ballots
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
    if (__ballot(valid && d == d0) == same) return same;
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const unsigned long long bb = __ballot((d >> bit) & 1u);
        same &= ((d >> bit) & 1u) ? bb : ~bb;
    }
    return same;
}

// Digit counts of one tile, each wave into counters of its own.  A round of
// 64 keys that share one digit (the high digits of keys that are nearly in
// order, as a batch's or a presorted fit's are) is counted by one add;
// other rounds by one LDS atomic per key.
__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t Q, int shift,
                                                           int64_t nb, uint32_t* __restrict__ hist)
{
    constexpr int WAVES = RS_THREADS / 64, PER_WAVE = RS_TILE / WAVES, WITEMS = PER_WAVE / 64;
    __shared__ uint32_t wcnt[WAVES][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) wcnt[k][tid] = 0;
    __syncthreads();
    const int64_t wbase = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * PER_WAVE;
    uint32_t key[WITEMS];
#pragma unroll
    for (int c = 0; c < WITEMS; ++c) {
        const int64_t e = wbase + c * 64 + lane;
        key[c] = e < Q ? keys[e] : 0u;
    }
#pragma unroll
    for (int c = 0; c < WITEMS; ++c) {
        const bool valid = wbase + c * 64 + lane < Q;
        const uint32_t d = (key[c] >> shift) & 255u;
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
        const unsigned long long vm = __ballot(valid);
        if (__ballot(valid && d == d0) == vm) {
            // lane 0 is valid whenever any lane is (the invalid keys end the
            // last tile); LDS accesses of one wave run in program order
            if (lane == 0 && vm) wcnt[w][d0] += (uint32_t)__popcll(vm);
        } else if (valid) {
            atomicAdd(&wcnt[w][d], 1u);
        }
    }
    __syncthreads();
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) sum += wcnt[k][tid];
    hist[(int64_t)tid * nb + blockIdx.x] = sum;
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

// Stable scatter of one digit pass.  Each wave ranks a contiguous quarter of
// the tile on its own (per-wave digit counters in LDS, no workgroup barrier
// per element round); the waves' counts then give every pair its position in
// the tile in (digit, input order) order, the pairs are placed in LDS and
// written out in that order: the keys of one digit leave as one run of
// consecutive positions (coalesced stores), not one scattered store per key.
__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                              const uint32_t* __restrict__ vin, int64_t Q, int shift,
                                                              int64_t nb, const uint32_t* __restrict__ offs,
                                                              uint32_t* __restrict__ kout, uint32_t* __restrict__ vout)
{
    static_assert(RS_THREADS == SC_THREADS, "one lane per digit in the tile's digit scan");
    constexpr int WAVES = RS_THREADS / 64, PER_WAVE = RS_TILE / WAVES, WITEMS = PER_WAVE / 64;
    __shared__ uint32_t wcnt[WAVES][256];  // per wave: digit counts, then the digit's first tile position
    __shared__ uint32_t gdelta[256];       // global position minus tile position, per digit
    __shared__ uint32_t scan_sh[SC_THREADS];
    __shared__ uint32_t tk[RS_TILE], tv[RS_TILE];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t blk = blockIdx.x;
    const int64_t t0 = blk * RS_TILE;
    const int n_here = (int)min((int64_t)RS_TILE, Q - t0);
#pragma unroll
    for (int k = 0; k < WAVES; ++k) wcnt[k][tid] = 0;
    __syncthreads();
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int64_t wbase = t0 + (int64_t)w * PER_WAVE;
    uint32_t key[WITEMS], val[WITEMS], rank[WITEMS];
#pragma unroll
    for (int c = 0; c < WITEMS; ++c) {
        const int64_t e = wbase + c * 64 + lane;
        const bool valid = e < Q;
        key[c] = valid ? kin[e] : 0u;
        val[c] = valid ? vin[e] : 0u;
    }
#pragma unroll
    for (int c = 0; c < WITEMS; ++c) {
        const bool valid = wbase + c * 64 + lane < Q;
        const uint32_t d = (key[c] >> shift) & 255u;
        const unsigned long long same = same_digit_lanes(d, valid);  // this wave's lanes of digit d
        const uint32_t r = (uint32_t)__popcll(same & lt);
        // a wave's LDS accesses run in program order: every lane reads the
        // count before the digit's first lane adds the round's lanes to it
        const uint32_t before = wcnt[w][d];
        rank[c] = before + r;
        if (valid && r == 0) wcnt[w][d] = before + (uint32_t)__popcll(same);
    }
    __syncthreads();
    // digit tid: its tile total, its first tile position, each wave's part
    uint32_t cw[WAVES], tot = 0;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) {
        cw[k] = wcnt[k][tid];
        tot += cw[k];
    }
    uint32_t tile_total;
    uint32_t at = block_excl_scan(tot, scan_sh, &tile_total);
    gdelta[tid] = offs[(int64_t)tid * nb + blk] - at;
#pragma unroll
    for (int k = 0; k < WAVES; ++k) {
        wcnt[k][tid] = at;
        at += cw[k];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < WITEMS; ++c) {
        if (wbase + c * 64 + lane < Q) {
            const uint32_t pos = wcnt[w][(key[c] >> shift) & 255u] + rank[c];
            tk[pos] = key[c];
            tv[pos] = val[c];
        }
    }
    __syncthreads();
    // tile positions 0..n_here-1 hold the tile's pairs in (digit, input
    // order) order; position p of digit d goes to gdelta[d] + p
    for (int p = tid; p < n_here; p += RS_THREADS) {
        const uint32_t k2 = tk[p];
        const uint32_t gpos = gdelta[(k2 >> shift) & 255u] + (uint32_t)p;
        kout[gpos] = k2;
        vout[gpos] = tv[p];
    }
}

// Cell starts: cs[c] = first sorted position whose key is >= c, for
// c = 0..n_cells (keys clamped to n_cells, the bucket of invalid directions).
// Sorted position i (0..Q) owns the cells c with key[i-1] < c <= key[i]
// (key[-1] = -1, key[Q] = n_cells): each cell has exactly one owner, so each
// entry is written once, without a search.  A wave writes the runs of its 64
// positions together, 64 consecutive cells per store; a run longer than
// CS_LONG cells, and the run of position Q (the cells after the last key),
// are listed and written by a workgroup each.  The list's order is free: the
// result is the same.
constexpr uint32_t CS_LONG = 65536;

// the cells [lo, hi] owned by sorted position i (lo > hi: none)
__device__ __forceinline__ void cs_owned(const uint32_t* __restrict__ sk, int64_t i, int64_t Q, uint32_t n_cells,
                                         uint32_t& lo, uint32_t& hi)
{
    lo = i > 0 ? min(sk[i - 1], n_cells) + 1u : 0u;
    hi = i < Q ? min(sk[i], n_cells) : n_cells;
}

__global__ __launch_bounds__(256) void k_cell_start(const uint32_t* __restrict__ sk, int64_t Q, uint32_t n_cells,
                                                    uint32_t* __restrict__ cs, uint32_t* __restrict__ n_long,
                                                    uint32_t* __restrict__ long_list)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    // both keys load at once (clamped indices, no branch)
    const uint32_t k_prev = sk[i > 0 ? min(i, Q) - 1 : 0], k_cur = sk[min(i, Q - 1)];
    uint32_t lo = i > 0 ? min(k_prev, n_cells) + 1u : 0u, hi = min(k_cur, n_cells);
    if (i >= Q) lo = 1, hi = 0;
    uint32_t count = hi >= lo ? hi - lo + 1u : 0u;
    if (count > CS_LONG) {
        long_list[atomicAdd(n_long, 1u)] = (uint32_t)i;
        count = 0;
    }
    // inclusive prefix of the counts over the wave
    uint32_t incl = count;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(incl, d);
        if (lane >= d) incl += o;
    }
    const uint32_t excl = incl - count;
    const uint32_t total = __shfl(incl, 63);  // at most 64 CS_LONG < 2^32
    const int64_t i_wave = i - lane;
    for (uint32_t t0 = 0; t0 < total; t0 += 64) {
        const uint32_t t = t0 + lane;
        // the owner: the last lane whose run starts at or before entry t
        int j = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1)
            if (__shfl(excl, j + step) <= t) j += step;
        const uint32_t e_j = __shfl(excl, j), lo_j = __shfl(lo, j);
        if (t < total) cs[lo_j + (t - e_j)] = (uint32_t)(i_wave + j);
    }
}

__global__ __launch_bounds__(256) void k_cell_start_long(const uint32_t* __restrict__ sk, int64_t Q, uint32_t n_cells,
                                                         uint32_t* __restrict__ cs, const uint32_t* __restrict__ n_long,
                                                         const uint32_t* __restrict__ long_list)
{
    const uint32_t n = *n_long;
    for (int64_t e = blockIdx.x; e <= (int64_t)n; e += gridDim.x) {
        const int64_t i = e < (int64_t)n ? (int64_t)long_list[e] : Q;
        uint32_t lo, hi;
        cs_owned(sk, i, Q, n_cells, lo, hi);
        for (int64_t c = (int64_t)lo + threadIdx.x; c <= (int64_t)hi; c += blockDim.x) cs[c] = (uint32_t)i;
    }
}

// ---------------------------------------------------------------------------
// Fused gradient pass.  One workgroup per tile of BT x BT texels of one face;
// its texels touch the BC x BC cells i0 in [p0-1, p0+BT-1], j0 in
// [q0-1, q0+BT-1].  In the sorted order each row of those cells is one
// contiguous range of queries, so the tile's queries are BC ranges, read as
// one concatenated list in rounds of BWD_THREADS:
//   * every lane takes the next query of the list (balanced, coalesced when
//     the directions are sorted) and computes its 16 weights (4 corners x 4
//     channels) into an LDS slot;
//   * every cell lane (one per cell) adds the slots of its segment, in
//     sorted order.
// Then each texel adds the corner sums of its <= 4 cells in a fixed order.
// Every sum has a fixed order: the result is deterministic, with no atomics.
//
// The fitting step (FIT) is the same pass with two changes: a query lane
// computes its upstream gradient itself (the forward query of the current
// LUT and the gradient of the value + normal objective, in place of reading
// grad_out), and each texel applies the Adam update to its summed gradient
// instead of writing it.  The updated texels go to a second LUT: a tile's
// halo queries read texels that neighbouring tiles update.
// ---------------------------------------------------------------------------
struct FitArgs {
    const float* tr;  // [Q] target radii
    const float* tn;  // [Q][3] target unit normals
    float w_value, inv_q;
    float4* lut_out;  // the updated LUT (never the input LUT)
    float4* m;        // Adam moments, LUT-shaped
    float4* v;
    AdamConsts k;
};

constexpr int BT = SHM_BWD_BT;
constexpr int BC = BT + 1;             // cells per tile side
// a tile with a cell of more than BWD_DENSE queries sums each round in runs
// of at most 16 slots (the serial per-cell loop would take one step per query)
constexpr int BWD_DENSE = 32;
constexpr int BWD_THREADS = BC * BC;
// dense tiles run in workgroups of BWD_GROUPS groups of BWD_THREADS lanes:
// group g takes rounds g, g + BWD_GROUPS, ... of the tile's list, and the
// groups' cell sums are added in group order at the end (a tile's list may
// hold a million queries: one group alone would make it the launch's tail)
constexpr int BWD_GROUPS = 4;
constexpr int BWD_DENSE_THREADS = BWD_THREADS * BWD_GROUPS;
constexpr int DIRS_THREADS = 256;      // lanes per workgroup of the direction gradient

// dL/d(16 footprint scalars) of one query, as 4 corners x (r, r_u h, r_v h, r_uv h^2).
// Each weight is gR Fs Ft + nlu Fs' Ft + nlv Fs Ft' for one s-basis function
// Fs (H0, H1, H0d, H1d at s) and one t-basis function Ft, so with
// P(Fs) = gR Fs + nlu Fs' and Qv(Fs) = nlv Fs it is P(Fs) Ft + Qv(Fs) Ft'.
__device__ __forceinline__ void query_weights(float gR, float nlu, float nlv, const Basis1& Sb, const Basis1& Tt,
                                              float4 w[4])
{
    // s-functions: value 0/1 (H0 = 1 - H1) and slope 0/1 (H0d, H1d), with derivatives
    const float sv[2] = {1.0f - Sb.h1, Sb.h1}, svd[2] = {-Sb.d1, Sb.d1};
    const float ss[2] = {Sb.h0d, Sb.h1d}, ssd[2] = {Sb.d0d, Sb.d1d};
    const float tv[2] = {1.0f - Tt.h1, Tt.h1}, tvd[2] = {-Tt.d1, Tt.d1};
    const float ts[2] = {Tt.h0d, Tt.h1d}, tsd[2] = {Tt.d0d, Tt.d1d};
#pragma unroll
    for (int cI = 0; cI < 2; ++cI) {
        const float Pv = gR * sv[cI] + nlu * svd[cI], Qv = nlv * sv[cI];
        const float Ps = gR * ss[cI] + nlu * ssd[cI], Qs = nlv * ss[cI];
#pragma unroll
        for (int cJ = 0; cJ < 2; ++cJ) {
            float4& o = w[cJ * 2 + cI];
            o.x = Pv * tv[cJ] + Qv * tvd[cJ];   // r
            o.y = Ps * tv[cJ] + Qs * tvd[cJ];   // r_u h
            o.z = Pv * ts[cJ] + Qv * tsd[cJ];   // r_v h
            o.w = Ps * ts[cJ] + Qs * tsd[cJ];   // r_uv h^2
        }
    }
}

// dL/d dirs of one query: second chart derivatives of the patch plus the
// derivative of the chart map (a = sc/ma, b = tc/ma) at d.  Its reciprocals
// and square root are the hardware's (~1 ulp): no decision depends on them.
template <bool FP16 = false>
__device__ __forceinline__ float3 dirs_grad(const void* __restrict__ lut_obj, int N, Loc L, float4 gq, float3 M,
                                         float3 S, float3 T, float x, float y, float z)
{
    const float Nf = (float)N;
    const float A = L.a, B = L.b;
    const float3 Sa = make_float3(S.x - A * M.x, S.y - A * M.y, S.z - A * M.z);
    const float3 Tb = make_float3(T.x - B * M.x, T.y - B * M.y, T.z - B * M.z);
    const float gS = gq.y * Sa.x + gq.z * Sa.y + gq.w * Sa.z;
    const float gT = gq.y * Tb.x + gq.z * Tb.y + gq.w * Tb.z;
    const float rho = __builtin_amdgcn_sqrtf(1.0f + A * A + B * B);
    const float kk2 = 0.5f * rho;
    const float gR = gq.x;
    const Foot F = load_foot<FP16, false>(lut_obj, N, L);
    const Patch2 Pp = hermite2(F, L.s, L.t);
    const float gM = gq.y * M.x + gq.z * M.y + gq.w * M.z;
    const float ru = Nf * Pp.rs, rv = Nf * Pp.rt;
    const float hN2 = 0.5f * Nf * Nf;
    const float common = (ru * gS + rv * gT) * __builtin_amdgcn_rcpf(2.0f * rho);
    const float dLda = 0.5f * Nf * gR * Pp.rs + A * common + kk2 * (hN2 * Pp.rss * gS - ru * gM + hN2 * Pp.rst * gT);
    const float dLdb = 0.5f * Nf * gR * Pp.rt + B * common + kk2 * (hN2 * Pp.rst * gS + hN2 * Pp.rtt * gT - rv * gM);
    const float im = __builtin_amdgcn_rcpf(x * M.x + y * M.y + z * M.z);
    return make_float3((dLda * Sa.x + dLdb * Tb.x) * im, (dLda * Sa.y + dLdb * Tb.y) * im,
                       (dLda * Sa.z + dLdb * Tb.z) * im);
}

// Workgroup barrier that orders LDS only: the threads of a tile exchange
// data through LDS alone, so the barrier need not wait for the global loads
// in flight (the next round's prefetch), as __syncthreads() would.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Where a texel tile sits: face size, face, first texel (p0, q0), the global
// index of the face's cell (0, 0) in the sorted keys, the global texel index
// of the face's texel (0, 0) in the LUT-shaped arrays, and the object's LUT.
struct TileGeo {
    int N, face, p0, q0;
    int64_t cbase, tex_base;
    const float* lut_obj;
};

// tile `tile` of n_obj uniform objects of face size N stored back to back
__device__ __forceinline__ TileGeo uniform_tile(int tile, int N, int tpf, const float* lut, int64_t lut_elems)
{
    const int C = N + 1, P = N + 2;
    const int per_face = tpf * tpf;
    const int64_t fo = tile / per_face;  // object * 6 + face
    const int b = tile - (int)(fo * per_face);
    TileGeo G;
    G.N = N;
    G.p0 = (b % tpf) * BT;
    G.q0 = (b / tpf) * BT;
    const int64_t obj = fo / 6;
    G.face = (int)(fo - obj * 6);
    G.cbase = fo * (int64_t)C * C;
    G.tex_base = fo * (int64_t)P * P;
    G.lut_obj = lut + obj * lut_elems;
    return G;
}

// One texel tile (workgroup-wide: every lane of the workgroup calls it with
// the same tile).  SORTED: dirs and gout hold the queries' directions and
// upstream gradients already in sorted order (read at the sorted position,
// coalesced); otherwise they are in query order and read through perm.
template <bool FIT, bool SORTED = false, bool DENSE = false>
__device__ __forceinline__ void bwd_tile(const TileGeo& G, const float* __restrict__ lut, int64_t Q,
                                         const float* __restrict__ dirs, const float* __restrict__ gout,
                                         const uint32_t* __restrict__ perm, const uint32_t* __restrict__ cs,
                                         float* __restrict__ grad_lut, const FitArgs& fa,
                                         const uint8_t* __restrict__ skip_flag = nullptr)
{
    // a tile another kernel handles (the dense ones) is left after the first
    // barrier: its flag loads beside the segment bounds, off the critical path
    const uint8_t skip = skip_flag != nullptr ? *skip_flag : 0;
    // one query's weights per lane, later the cell sums: corner-major, so that
    // the 16-byte accesses of consecutive lanes fall on consecutive banks
    // dense tiles pad each corner's row by one float4 every 16 slots (and
    // the rows by 4): the run sums below then read 64 distinct banks per wave
    constexpr int SROW = DENSE ? BWD_THREADS + BWD_THREADS / 16 + 4 : BWD_THREADS;
    constexpr int GS = DENSE ? BWD_GROUPS : 1;  // lane groups of BWD_THREADS
    __shared__ float4 slot_m[GS * 4 * SROW];
    const int tid = threadIdx.x;
    const int grp = DENSE ? tid / BWD_THREADS : 0, lt = DENSE ? tid % BWD_THREADS : tid;
    auto slot_of = [&](int gg, int k, int s) -> float4& {
        return slot_m[(gg * 4 + k) * SROW + (DENSE ? s + (s >> 4) : s)];
    };
    auto slot = [&](int k, int s) -> float4& { return slot_of(grp, k, s); };
    // sorted positions and list offsets are below Q < 2^32 - 1: 32 bits
    __shared__ uint32_t row_start[BC];       // first sorted position of each cell row's range
    __shared__ uint32_t row_len[BC];         // queries in each cell row's range
    __shared__ uint32_t row_off[BC + 1];     // offsets of the rows in the concatenated list
    __shared__ uint64_t run_end[DENSE ? GS * BWD_THREADS / 64 : 1];  // dense tiles: per wave, the slots that end a run
    const int N = G.N;
    const int C = N + 1, P = N + 2;
    const int p0 = G.p0, q0 = G.q0;
    const int face = G.face;
    const int64_t cbase = G.cbase;
    const int i_lo = max(p0 - 1, 0), i_hi = min(p0 + BT - 1, N);  // the tile's cell columns (p0 <= N + 1)
    // this lane's cell: its segment bounds load beside the row setup (every
    // group of a dense tile accumulates its own rounds' sums per cell)
    const int ci = lt % BC, cj = lt / BC;
    const int i0c = p0 - 1 + ci, j0c = q0 - 1 + cj;
    // with no queries the sort wrote no segment starts: every list is empty
    const bool cell_ok = Q > 0 && i0c >= 0 && i0c <= N && j0c >= 0 && j0c <= N;
    const uint32_t Qu = (uint32_t)Q;
    uint32_t cs_lo = 0, cs_hi = 0;
    if (cell_ok) {
        const int64_t c = cbase + (int64_t)j0c * C + i0c;
        cs_lo = cs[c];
        cs_hi = cs[c + 1];
    }
    if (tid < BC) {
        const int j0 = q0 - 1 + tid;
        uint32_t a = 0, e = 0;
        if (Q > 0 && j0 >= 0 && j0 <= N) {
            const int64_t c0 = cbase + (int64_t)j0 * C;
            a = min(cs[c0 + i_lo], Qu);
            e = min(max(cs[c0 + i_hi + 1], a), Qu);
        }
        row_start[tid] = a;
        row_len[tid] = e - a;
    }
    lds_barrier();
    if (skip) return;  // uniform over the workgroup
    if (tid <= BC) {  // exclusive prefix: independent reads, no serial chain
        uint32_t o = 0;
        for (int k = 0; k < tid; ++k) o += row_len[k];
        row_off[tid] = o;
    }
    lds_barrier();
    uint32_t seg_lo = 0, seg_hi = 0;
    if (cell_ok) {
        const uint32_t rs = row_start[cj], len = row_off[cj + 1] - row_off[cj];
        const uint32_t a = min(cs_lo > rs ? cs_lo - rs : 0u, len);
        const uint32_t e = min(max(cs_hi > rs ? cs_hi - rs : 0u, a), len);
        seg_lo = row_off[cj] + a;
        seg_hi = row_off[cj] + e;
    }
    const uint32_t total = row_off[BC];
    const float Nf = (float)N;
    float3 M, S, T;
    frame_of(face, M, S, T);
    float4 acc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    // the query at list position g and its cell row (binary search for the
    // last row starting at or before g: empty rows share their successor's
    // offset, so it lands on the row holding g).  The permutation is read at
    // a position clamped into the list and the entry past the end is marked
    // by the flag alone: no branch, so the loaded index is not waited for
    // until its first use, a round's weights later.
    auto query_at = [&](int64_t g, int& r, bool& valid) -> uint32_t {
        valid = g < (int64_t)total;
        const uint32_t gc = valid ? (uint32_t)g : total - 1;
        r = 0;
#pragma unroll
        for (int step = BC / 2; step >= 1; step >>= 1)
            if (row_off[r + step] <= gc) r += step;
        const uint32_t pos = min(row_start[r] + (gc - row_off[r]), Qu - 1);
        if constexpr (SORTED) return pos;
        else return perm[pos];
    };
    // the upstream gradient of query q, or for the fitting step its targets
    // (R*, n*), from which the lane computes the upstream gradient
    auto upstream_in = [&](int64_t q) -> float4 {
        if constexpr (FIT) return make_float4(fa.tr[q], fa.tn[3 * q], fa.tn[3 * q + 1], fa.tn[3 * q + 2]);
        else return reinterpret_cast<const float4*>(gout)[q];
    };
    static_assert(!(FIT && SORTED), "the fitting step reads its inputs in query order");
    const float* lut_obj = G.lut_obj;
    // software pipeline: round k + 1's index, direction and upstream
    // gradient loads are in flight while round k computes and reduces
    // (an empty list, as with no queries at all, loads nothing: its clamped
    // position would not name a query)
    int r_cur = 0;
    bool v_cur = false;
    uint32_t q_cur = 0;
    float x = 0.0f, y = 0.0f, z = 0.0f;
    float4 gq = make_float4(0.f, 0.f, 0.f, 0.f);
    // this group's rounds start at list position grp * BWD_THREADS and step
    // by GS * BWD_THREADS; every group runs every round's barriers
    constexpr int STEP = GS * BWD_THREADS;
    const int64_t gofs = (int64_t)grp * BWD_THREADS;
    if (total > 0) {
        q_cur = query_at(gofs + lt, r_cur, v_cur);
        x = dirs[3 * (size_t)q_cur];
        y = dirs[3 * (size_t)q_cur + 1];
        z = dirs[3 * (size_t)q_cur + 2];
        gq = upstream_in(q_cur);
    }
    for (int64_t base0 = 0; base0 < total; base0 += STEP) {
        const int64_t base = base0 + gofs;  // this group's round
        int r_next;
        bool v_next;
        const uint32_t q_next = query_at(base + STEP + lt, r_next, v_next);
        // list positions base + lt < total hold a query and fill their
        // slot; the reduction below reads no other slot
        int my_cell = -1;  // dense tiles: the tile cell of this lane's query, -1 for none
        if (v_cur) {
            const Loc L = locate(x, y, z, N);  // the cell of row r_cur (keys come from the same decision)
            if constexpr (FIT) {
                // the forward query and the objective's gradient with respect
                // to its output
                gq = loss_grad_one(fit_forward(lut_obj, N, L), x, y, z, gq.x, gq.y, gq.z, gq.w, fa.w_value, fa.inv_q);
            }
            {
                const float A = L.a, B = L.b;
                const float gS = gq.y * (S.x - A * M.x) + gq.z * (S.y - A * M.y) + gq.w * (S.z - A * M.z);
                const float gT = gq.y * (T.x - B * M.x) + gq.z * (T.y - B * M.y) + gq.w * (T.z - B * M.z);
                const float kk2 = 0.5f * __builtin_amdgcn_sqrtf(1.0f + A * A + B * B);
                float4 w[4];
                query_weights(gq.x, Nf * kk2 * gS, Nf * kk2 * gT, basis1(L.s), basis1(L.t), w);
#pragma unroll
                for (int k = 0; k < 4; ++k) slot(k, lt) = w[k];
            }
            if constexpr (DENSE) my_cell = r_cur * BC + (L.i0 - (p0 - 1));
        }
        if constexpr (DENSE) {
            // slot lt ends a run when the next slot holds another cell (or
            // none) or a chunk of 16 slots ends; chunks do not cross waves
            const int nb = __shfl_down(my_cell, 1);
            const uint64_t m = __ballot((lt & 15) == 15 || nb != my_cell);
            if ((lt & 63) == 0) run_end[grp * (BWD_THREADS / 64) + (lt >> 6)] = m;
        }
        // unconditional: q_next is a valid index even past the list's end
        x = dirs[3 * (size_t)q_next];
        y = dirs[3 * (size_t)q_next + 1];
        z = dirs[3 * (size_t)q_next + 2];
        gq = upstream_in(q_next);
        q_cur = q_next;
        r_cur = r_next;
        v_cur = v_next;
        {
            lds_barrier();
            // the segment's slots in this group's round (base may pass the
            // list's end, then the range is empty; base < 2^32 + STEP)
            const uint32_t b = base < (int64_t)total ? (uint32_t)base : total;
            const int lo = (int)min(seg_lo > b ? seg_lo - b : 0u, (uint32_t)BWD_THREADS);
            const int hi = (int)min(seg_hi > b ? seg_hi - b : 0u, (uint32_t)BWD_THREADS);
            if constexpr (!DENSE) {
                for (int k2 = lo; k2 < hi; ++k2) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float4 v = slot(k, k2);
                        acc[k].x += v.x;
                        acc[k].y += v.y;
                        acc[k].z += v.z;
                        acc[k].w += v.w;
                    }
                }
            } else {
                // a cell's segment may fill whole rounds: first each run of
                // one cell inside a chunk of 16 slots is summed in order, one
                // lane per (chunk, scalar), into the run's last slot; then
                // each cell lane adds its runs' sums in order (at most one
                // per chunk instead of one per query)
                {
                    const int chunk = lt >> 4, ch = lt & 15;
                    float* col = reinterpret_cast<float*>(&slot(ch >> 2, chunk * 16)) + (ch & 3);
                    const uint32_t ends =
                        (uint32_t)(run_end[grp * (BWD_THREADS / 64) + (chunk >> 2)] >> ((chunk & 3) * 16));
                    float v[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i) v[i] = col[4 * i];
                    // the running sum is stored at every slot; only the run
                    // ends are read
                    float run = 0.0f;
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        run += v[i];
                        col[4 * i] = run;
                        run = ((ends >> i) & 1u) ? 0.0f : run;
                    }
                }
                lds_barrier();
                for (int p = lo; p < hi;) {
                    const int pe = min(hi, (p | 15) + 1) - 1;  // the end of the run holding p
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float4 v = slot(k, pe);
                        acc[k].x += v.x;
                        acc[k].y += v.y;
                        acc[k].z += v.z;
                        acc[k].w += v.w;
                    }
                    p = pe + 1;
                }
            }
            lds_barrier();
        }
    }
    // the fitting step's parameters and moments of this lane's texel load
    // while the cell sums are exchanged
    const int t_x = tid % BT, t_y = tid / BT, t_p = p0 + t_x, t_q = q0 + t_y;
    const bool t_ok = tid < BT * BT && t_p <= N + 1 && t_q <= N + 1;
    const int64_t t_i = G.tex_base + (int64_t)t_q * P + t_p;
    float4 pp, mm, vv;
    if (FIT && t_ok) {
        pp = reinterpret_cast<const float4*>(lut)[t_i];
        mm = fa.m[t_i];
        vv = fa.v[t_i];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) slot(k, lt) = acc[k];
    lds_barrier();
    if constexpr (DENSE) {
        // the groups' cell sums, added in group order into group 0's slots
        if (grp == 0) {
#pragma unroll
            for (int gg = 1; gg < GS; ++gg)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float4 v = slot_of(gg, k, lt);
                    acc[k].x += v.x;
                    acc[k].y += v.y;
                    acc[k].z += v.z;
                    acc[k].w += v.w;
                }
#pragma unroll
            for (int k = 0; k < 4; ++k) slot(k, lt) = acc[k];
        }
        lds_barrier();
    }
    // texel (p0 + tx, q0 + ty) is corner (1,1) of cell (tx, ty), (0,1) of
    // (tx+1, ty), (1,0) of (tx, ty+1) and (0,0) of (tx+1, ty+1) in tile cells
    static_assert(BT * BT <= BWD_THREADS, "one texel per lane");
    if (t_ok) {
        const int tx = t_x, ty = t_y;
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int dj = 1; dj >= 0; --dj)
#pragma unroll
            for (int di = 1; di >= 0; --di) {
                const float4 v = slot(dj * 2 + di, (ty + 1 - dj) * BC + (tx + 1 - di));
                a.x += v.x;
                a.y += v.y;
                a.z += v.z;
                a.w += v.w;
            }
        if constexpr (FIT) {
            adam_texel(pp, a, mm, vv, fa.k);
            fa.lut_out[t_i] = pp;
            fa.m[t_i] = mm;
            fa.v[t_i] = vv;
        } else {
            reinterpret_cast<float4*>(grad_lut)[t_i] = a;
        }
    }
}

// Whether a tile is dense (some cell of its 16 x 16 cells holds more than
// BWD_DENSE queries): decided once per sort, so that each backward runs the
// sparse and the dense tiles in two kernels of their own (the dense sums need
// registers the sparse kernel should not pay for).
__device__ __forceinline__ void tile_dense_flag(const TileGeo& G, const uint32_t* __restrict__ cs, DenseTiles D,
                                                uint32_t t)
{
    // one wave per tile, BC * BC / 64 of its cells per lane
    static_assert(BC * BC % 64 == 0, "whole cells per lane");
    const int lane = threadIdx.x & 63;
    const int C = G.N + 1;
    bool dense = false;
#pragma unroll
    for (int k = 0; k < BC * BC / 64; ++k) {
        const int cell = lane + 64 * k;
        const int i0c = G.p0 - 1 + cell % BC, j0c = G.q0 - 1 + cell / BC;
        if (i0c >= 0 && i0c <= G.N && j0c >= 0 && j0c <= G.N) {
            const int64_t c = G.cbase + (int64_t)j0c * C + i0c;
            dense |= (int64_t)cs[c + 1] - cs[c] > BWD_DENSE;
        }
    }
    const bool any = __ballot(dense) != 0;
    if (lane == 0) {
        D.flag[t] = any ? 1 : 0;
        if (any) D.list[atomicAdd(D.count, 1u)] = t;  // integer atomic: the list's order is free
    }
}

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

// workgroups of a dense-tile kernel whose tile count the host does not know:
// one per compute unit (a launch that finds no dense tile stays cheap), at
// most one per tile
static inline int64_t dense_grid(int64_t n_tiles)
{
    return std::max<int64_t>(1, std::min<int64_t>(n_tiles, (int64_t)device_cu_count()));
}

// tile flags: one wave per tile, 4 tiles per workgroup of 256
__global__ __launch_bounds__(256) void k_tile_dense(int N, int tiles_per_face, int64_t n_tiles,
                                                    const uint32_t* __restrict__ cs, DenseTiles D)
{
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= n_tiles) return;
    tile_dense_flag(uniform_tile((int)t, N, tiles_per_face, nullptr, 0), cs, D, (uint32_t)t);
}

// cell starts from the sorted keys sk (Q > 0); the radix histogram's first
// word counts the long runs and the key buffer not holding sk lists them
// (the list holds at most Q positions)
static void launch_cell_start(const BwdLayout& W, char* base, const uint32_t* sk, hipStream_t stream)
{
    uint32_t* cs = reinterpret_cast<uint32_t*>(base + W.cstart);
    uint32_t* n_long = reinterpret_cast<uint32_t*>(base + W.hist);
    uint32_t* k_free = reinterpret_cast<uint32_t*>(base + (sk == reinterpret_cast<const uint32_t*>(base + W.keys0)
                                                                 ? W.keys1
                                                                 : W.keys0));
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, stream, n_long, 0u);
    hipLaunchKernelGGL(k_cell_start, dim3((unsigned)((W.Q + 255) / 256)), dim3(256), 0, stream, sk, W.Q,
                       (uint32_t)W.n_cells, cs, n_long, k_free);
    hipLaunchKernelGGL(k_cell_start_long, dim3((unsigned)(4 * device_cu_count())), dim3(256), 0, stream, sk, W.Q,
                       (uint32_t)W.n_cells, cs, (const uint32_t*)n_long, (const uint32_t*)k_free);
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
    launch_cell_start(W, base, k0, stream);
    const uint32_t* cs = reinterpret_cast<const uint32_t*>(base + W.cstart);
    if (W.n_tiles > 0) {
        const DenseTiles D = dense_tiles(base + W.dense, W.n_tiles);
        hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, stream, D.count, 0u);
        hipLaunchKernelGGL(k_tile_dense, dim3((unsigned)((W.n_tiles + 3) / 4)), dim3(256), 0, stream, N,
                           (N + 2 + BT - 1) / BT, W.n_tiles, (const uint32_t*)cs, D);
    }
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

// the sparse tiles, one workgroup per tile (a dense tile's workgroup exits)
template <bool FIT>
__global__ __launch_bounds__(BWD_THREADS) void k_bwd_fused(const float* __restrict__ lut, int N, int64_t lut_elems,
                                                           int64_t Q, const float* __restrict__ dirs,
                                                           const float* __restrict__ gout,
                                                           const uint32_t* __restrict__ perm,
                                                           const uint32_t* __restrict__ cs, int tiles_per_face,
                                                           const uint8_t* __restrict__ dense_flag,
                                                           float* __restrict__ grad_lut, FitArgs fa)
{
    bwd_tile<FIT>(uniform_tile((int)blockIdx.x, N, tiles_per_face, lut, lut_elems), lut, Q, dirs, gout, perm, cs,
                  grad_lut, fa, dense_flag != nullptr ? dense_flag + blockIdx.x : nullptr);
}

// the dense tiles, from the sort's list: a small persistent grid, so that a
// backward without dense tiles pays little for this launch
template <bool FIT>
__global__ __launch_bounds__(BWD_DENSE_THREADS) void k_bwd_fused_dense(const float* __restrict__ lut, int N,
                                                                 int64_t lut_elems, int64_t Q,
                                                                 const float* __restrict__ dirs,
                                                                 const float* __restrict__ gout,
                                                                 const uint32_t* __restrict__ perm,
                                                                 const uint32_t* __restrict__ cs, int tiles_per_face,
                                                                 const uint32_t* __restrict__ count,
                                                                 const uint32_t* __restrict__ list,
                                                                 float* __restrict__ grad_lut, FitArgs fa)
{
    const uint32_t n = *count;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        bwd_tile<FIT, false, true>(uniform_tile((int)list[i], N, tiles_per_face, lut, lut_elems), lut, Q, dirs, gout,
                                   perm, cs, grad_lut, fa);
        lds_barrier();  // the next tile reuses the workgroup's LDS
    }
}

// Direction gradients of DIRS_THREADS consecutive queries (block blk), in the
// queries' own order: a direction's gradient involves no other query, so it
// needs neither the sort nor LDS.  NaN for an invalid direction.
//
// The object of query q is floor(q / q_per_obj), taken without a division:
// for q < 2^32 and 2 <= d < 2^32, m = floor((2^64 - 1) / d) + 1 exceeds
// 2^64 / d by at most 1 (d a power of two: by 0), so q m / 2^64 exceeds q / d
// by less than q / 2^64 < 1 / d, too little to reach the next integer; its
// integer part (the high word of the product) is floor(q / d).  d = 1 is
// passed as m = 0.
__device__ __forceinline__ void bwd_dirs_block(int64_t blk, const float* __restrict__ lut, int N, int64_t lut_elems,
                                               int64_t Q, uint64_t obj_magic, const float* __restrict__ dirs,
                                               const float* __restrict__ gout, float* __restrict__ grad_dirs)
{
    const int64_t q = blk * DIRS_THREADS + threadIdx.x;
    if (q >= Q) return;
    const uint64_t obj = obj_magic == 0 ? (uint64_t)q : __umul64hi((uint64_t)q, obj_magic);
    const float x = dirs[3 * q], y = dirs[3 * q + 1], z = dirs[3 * q + 2];
    const Loc L = locate(x, y, z, N);
    float3 gd;
    if (L.face < 0) {
        const float nan = __builtin_nanf("");
        gd = make_float3(nan, nan, nan);
    } else {
        const float4 gq = reinterpret_cast<const float4*>(gout)[q];
        float3 M, S, T;
        frame_of(L.face, M, S, T);
        gd = dirs_grad(lut + (int64_t)obj * lut_elems, N, L, gq, M, S, T, x, y, z);
    }
    grad_dirs[3 * q] = gd.x;
    grad_dirs[3 * q + 1] = gd.y;
    grad_dirs[3 * q + 2] = gd.z;
}

__global__ __launch_bounds__(DIRS_THREADS) void k_bwd_dirs(const float* __restrict__ lut, int N, int64_t lut_elems,
                                                          int64_t Q, uint64_t obj_magic, const float* __restrict__ dirs,
                                                          const float* __restrict__ gout,
                                                          float* __restrict__ grad_dirs)
{
    bwd_dirs_block(blockIdx.x, lut, N, lut_elems, Q, obj_magic, dirs, gout, grad_dirs);
}

// the multiplier of bwd_dirs_block for d queries per object (1 <= d < 2^32)
static uint64_t obj_magic(int64_t d)
{
    return d <= 1 ? 0 : UINT64_MAX / (uint64_t)d + 1;
}

__global__ void k_zero_f4(float4* __restrict__ a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// ---------------------------------------------------------------------------
// Backward of a plan's objects: face sizes, LUT offsets and query ranges of
// their own.  The host builds three prefix arrays over the objects (n_obj + 1
// entries each): the first global cell key of each object (cells of the
// objects before it), its first LUT-gradient tile (6 tpf^2 per object) and
// its first query tile (OBJ_QT queries).  A workgroup finds its object by
// binary search over the prefix of its kind; everything else is the uniform
// path's arithmetic, so a plan's backward gives each object the bits of a
// one-object backward of that object's queries.
// ---------------------------------------------------------------------------
constexpr int OBJ_QT = 256;  // queries per query tile

struct BwdObjects {
    const shm_object* objs;
    const int64_t* cell_base;
    const int64_t* tile_base;
    const int64_t* qtile_base;
    const int32_t* tile_obj;   // object of each LUT-gradient tile
    const int32_t* qtile_obj;  // object of each query tile
    int64_t n_obj;
};

__global__ void k_keys_init(int64_t Q, uint32_t invalid_key, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= Q) return;
    keys[q] = invalid_key;
    vals[q] = (uint32_t)q;
}

__global__ __launch_bounds__(OBJ_QT) void k_cell_keys_objects(BwdObjects B, const float* __restrict__ dirs,
                                                              uint32_t invalid_key, uint32_t* __restrict__ keys)
{
    const int64_t t = blockIdx.x;
    const int64_t o = B.qtile_obj[t];
    const shm_object ob = B.objs[o];
    const int64_t k = (t - B.qtile_base[o]) * OBJ_QT + threadIdx.x;
    if (k >= ob.q_count) return;
    const int64_t q = ob.q_begin + k;
    const Loc L = locate(dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2], ob.N);
    const int64_t C = ob.N + 1;
    keys[q] = L.face < 0 ? invalid_key : (uint32_t)(B.cell_base[o] + ((int64_t)L.face * C + L.j0) * C + L.i0);
}

// row i of dst = row perm[i] of src (rows of W floats): the queries' inputs
// in sorted order, read at random once so that the tiles read them coalesced.
// Each XCD takes a contiguous eighth of the rows: an object's rows, and so
// the random reads of its source rows, stay on one XCD and its L2.
template <int W>
__global__ void k_gather_rows(const uint32_t* __restrict__ perm, const float* __restrict__ src, int64_t Q,
                              float* __restrict__ dst)
{
    const int64_t i = (int64_t)xcd_remap((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= Q) return;
    const int64_t q = perm[i];
    if constexpr (W == 4) {
        reinterpret_cast<float4*>(dst)[i] = reinterpret_cast<const float4*>(src)[q];
    } else {
#pragma unroll
        for (int k = 0; k < W; ++k) dst[W * i + k] = src[W * q + k];
    }
}

// tile t of a plan's objects
__device__ __forceinline__ TileGeo object_tile(const BwdObjects& B, int64_t t)
{
    const int64_t o = B.tile_obj[t];
    const shm_object ob = B.objs[o];
    const int N = ob.N, C = N + 1, P = N + 2;
    const int tpf = (P + BT - 1) / BT, per_face = tpf * tpf;
    const int local = (int)(t - B.tile_base[o]);
    TileGeo G;
    G.N = N;
    G.face = local / per_face;
    const int b = local - G.face * per_face;
    G.p0 = (b % tpf) * BT;
    G.q0 = (b / tpf) * BT;
    G.cbase = B.cell_base[o] + (int64_t)G.face * C * C;
    G.tex_base = ob.lut_offset / 4 + (int64_t)G.face * P * P;  // texels of 4 elements
    G.lut_obj = nullptr;                                       // read only by the fitting step
    return G;
}

// A plan tile's geometry and kind, written once per sort so that the tile
// kernels start from one (scalar) load instead of the chain tile -> object
// -> object record -> divisions.  kind: 0 no query in the tile's cells (a
// zero gradient), 1 sparse, 2 dense (some cell with more than BWD_DENSE).
struct TileRec {
    int32_t N, face_kind, p0, q0;  // face_kind = face | kind << 8
    int64_t cbase, tex_base;
};
static_assert(sizeof(TileRec) == 32, "one 32-byte record per tile");

__device__ __forceinline__ TileGeo tile_of_rec(const TileRec& r)
{
    TileGeo G;
    G.N = r.N;
    G.face = r.face_kind & 255;
    G.p0 = r.p0;
    G.q0 = r.q0;
    G.cbase = r.cbase;
    G.tex_base = r.tex_base;
    G.lut_obj = nullptr;
    return G;
}

__global__ __launch_bounds__(256) void k_tile_dense_objects(BwdObjects B, int64_t n_tiles,
                                                            const uint32_t* __restrict__ cs, DenseTiles D,
                                                            TileRec* __restrict__ recs)
{
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= n_tiles) return;
    const TileGeo G = object_tile(B, t);
    const int lane = threadIdx.x & 63;
    const int C = G.N + 1;
    bool dense = false, any = false;
#pragma unroll
    for (int k = 0; k < BC * BC / 64; ++k) {
        const int cell = lane + 64 * k;
        const int i0c = G.p0 - 1 + cell % BC, j0c = G.q0 - 1 + cell / BC;
        if (i0c >= 0 && i0c <= G.N && j0c >= 0 && j0c <= G.N) {
            const int64_t c = G.cbase + (int64_t)j0c * C + i0c;
            const int64_t n = (int64_t)cs[c + 1] - cs[c];
            dense |= n > BWD_DENSE;
            any |= n > 0;
        }
    }
    const bool d = __ballot(dense) != 0, a = __ballot(any) != 0;
    if (lane == 0) {
        D.flag[t] = d ? 1 : 0;
        if (d) D.list[atomicAdd(D.count, 1u)] = (uint32_t)t;  // integer atomic: the list's order is free
        TileRec r;
        r.N = G.N;
        r.face_kind = G.face | ((d ? 2 : (a ? 1 : 0)) << 8);
        r.p0 = G.p0;
        r.q0 = G.q0;
        r.cbase = G.cbase;
        r.tex_base = G.tex_base;
        recs[t] = r;
    }
}

// recs: the tile records of the sort; null when there are no queries (every
// tile then has a zero gradient, its geometry taken from the objects)
__global__ __launch_bounds__(BWD_THREADS) void k_bwd_fused_objects(BwdObjects B, const TileRec* __restrict__ recs,
                                                                   int64_t Q, const float* __restrict__ sdirs,
                                                                   const float* __restrict__ sgout,
                                                                   const uint32_t* __restrict__ perm,
                                                                   const uint32_t* __restrict__ cs,
                                                                   float* __restrict__ grad_lut)
{
    const int64_t t = blockIdx.x;
    TileGeo G;
    int kind = 0;
    if (recs != nullptr) {
        const TileRec r = recs[t];
        G = tile_of_rec(r);
        kind = r.face_kind >> 8;
    } else {
        G = object_tile(B, t);
    }
    if (kind == 2) return;  // a dense tile: k_bwd_fused_objects_dense
    if (kind == 0) {        // no query in the tile's cells: a zero gradient, without the row setup
        const int P = G.N + 2;
        const int tid = threadIdx.x, t_x = tid % BT, t_y = tid / BT;
        if (tid < BT * BT && G.p0 + t_x <= G.N + 1 && G.q0 + t_y <= G.N + 1)
            reinterpret_cast<float4*>(grad_lut)[G.tex_base + (int64_t)(G.q0 + t_y) * P + G.p0 + t_x] =
                make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    bwd_tile<false, true>(G, nullptr, Q, sdirs, sgout, perm, cs, grad_lut, FitArgs{});
}

__global__ __launch_bounds__(BWD_DENSE_THREADS) void k_bwd_fused_objects_dense(const TileRec* __restrict__ recs, int64_t Q,
                                                                         const float* __restrict__ sdirs,
                                                                         const float* __restrict__ sgout,
                                                                         const uint32_t* __restrict__ perm,
                                                                         const uint32_t* __restrict__ cs,
                                                                         const uint32_t* __restrict__ count,
                                                                         const uint32_t* __restrict__ list,
                                                                         float* __restrict__ grad_lut)
{
    const uint32_t n = *count;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        bwd_tile<false, true, true>(tile_of_rec(recs[list[i]]), nullptr, Q, sdirs, sgout, perm, cs, grad_lut,
                                    FitArgs{});
        lds_barrier();  // the next tile reuses the workgroup's LDS
    }
}

template <bool FP16>
__global__ __launch_bounds__(OBJ_QT) void k_bwd_dirs_objects(BwdObjects B, const void* __restrict__ lut,
                                                             const float* __restrict__ dirs,
                                                             const float* __restrict__ gout,
                                                             float* __restrict__ grad_dirs)
{
    // an object's query tiles are contiguous: on one XCD, its LUT stays in that L2
    const int64_t t = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int64_t o = B.qtile_obj[t];
    const shm_object ob = B.objs[o];
    const int64_t k = (t - B.qtile_base[o]) * OBJ_QT + threadIdx.x;
    if (k >= ob.q_count) return;
    const int64_t q = ob.q_begin + k;
    const float x = dirs[3 * q], y = dirs[3 * q + 1], z = dirs[3 * q + 2];
    const Loc L = locate(x, y, z, ob.N);
    float3 gd;
    if (L.face < 0) {
        const float nan = __builtin_nanf("");
        gd = make_float3(nan, nan, nan);
    } else {
        const float4 gq = reinterpret_cast<const float4*>(gout)[q];
        float3 M, S, T;
        frame_of(L.face, M, S, T);
        const char* base = reinterpret_cast<const char*>(lut) + (size_t)ob.lut_offset * (FP16 ? 2 : 4);
        gd = dirs_grad<FP16>(base, ob.N, L, gq, M, S, T, x, y, z);
    }
    grad_dirs[3 * q] = gd.x;
    grad_dirs[3 * q + 1] = gd.y;
    grad_dirs[3 * q + 2] = gd.z;
}

// Sort of a plan's queries: Q rows (rows outside every object keep the
// invalid key and sort last), n_cells keys.  The workspace layout is the
// uniform one for (Q, n_cells).
static BwdLayout bwd_layout_cells(int64_t Q, int64_t n_cells, int64_t n_tiles)
{
    BwdLayout W;
    W.n_tiles = n_tiles;
    W.Q = Q;
    W.n_cells = n_cells;
    W.nb = (W.Q + RS_TILE - 1) / RS_TILE;
    int bits = 1;
    while (((int64_t)1 << bits) <= W.n_cells) ++bits;
    W.passes = (bits + 7) / 8;
    size_t at = 0;
    auto take = [&](size_t bytes) { size_t a = at; at += align256(bytes); return a; };
    W.keys0 = take(W.Q * 4);
    W.vals0 = take(W.Q * 4);
    W.keys1 = take(W.Q * 4);
    W.vals1 = take(W.Q * 4);
    W.cstart = take((W.n_cells + 1) * 4);
    W.hist = take((size_t)256 * W.nb * 4);
    W.tsum = take(((size_t)256 * W.nb + SC_TILE - 1) / SC_TILE * 4);
    W.sdirs = take(W.Q * 12);  // directions in sorted order (with the sort)
    W.sgout = take(W.Q * 16);  // upstream gradients in sorted order (per backward)
    W.dense = take(dense_bytes(n_tiles));
    W.geo = take((size_t)n_tiles * 32);  // each tile's geometry and kind (TileRec), with the sort
    W.total = at;
    return W;
}

size_t backward_objects_workspace_bytes(int64_t Q, int64_t n_cells, int64_t n_tiles)
{
    return bwd_layout_cells(Q, n_cells, n_tiles).total;
}
int backward_tile_texels() { return BT; }
int backward_query_tile() { return OBJ_QT; }

static void radix_sort_pass_all(const BwdLayout& W, char* base, hipStream_t stream, uint32_t*& k0, uint32_t*& v0)
{
    uint32_t* k1 = reinterpret_cast<uint32_t*>(base + W.keys1);
    uint32_t* v1 = reinterpret_cast<uint32_t*>(base + W.vals1);
    uint32_t* hist = reinterpret_cast<uint32_t*>(base + W.hist);
    uint32_t* tsum = reinterpret_cast<uint32_t*>(base + W.tsum);
    const int64_t n_hist = (int64_t)256 * W.nb;
    const int64_t n_tiles = (n_hist + SC_TILE - 1) / SC_TILE;
    for (int p = 0; p < W.passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)W.nb), dim3(RS_THREADS), 0, stream, k0, W.Q, shift, W.nb, hist);
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)n_tiles), dim3(SC_THREADS), 0, stream, hist, n_hist, tsum);
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SC_THREADS), 0, stream, tsum, n_tiles);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)n_tiles), dim3(SC_THREADS), 0, stream, hist, n_hist, tsum);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)W.nb), dim3(RS_THREADS), 0, stream, k0, v0, W.Q, shift, W.nb,
                           hist, k1, v1);
        uint32_t* t = k0; k0 = k1; k1 = t;
        t = v0; v0 = v1; v1 = t;
    }
}

const uint32_t* backward_objects_dense_count(const BwdObjectsHost& H, const void* ws)
{
    const BwdLayout W = bwd_layout_cells(H.Q, H.n_cells, H.n_tiles);
    return reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(ws) + W.dense);
}

int launch_backward_sort_objects(const BwdObjectsHost& H, const float* dirs, void* ws, hipStream_t stream)
{
    const BwdLayout W = bwd_layout_cells(H.Q, H.n_cells, H.n_tiles);
    if (W.Q == 0) return SHM_OK;
    char* base = reinterpret_cast<char*>(ws);
    uint32_t* k0 = reinterpret_cast<uint32_t*>(base + W.keys0);
    uint32_t* v0 = reinterpret_cast<uint32_t*>(base + W.vals0);
    const BwdObjects B{H.objs, H.cell_base, H.tile_base, H.qtile_base, H.tile_obj, H.qtile_obj, H.n_obj};
    hipLaunchKernelGGL(k_keys_init, dim3((unsigned)((W.Q + 255) / 256)), dim3(256), 0, stream, W.Q,
                       (uint32_t)W.n_cells, k0, v0);
    if (H.n_qtiles > 0)
        hipLaunchKernelGGL(k_cell_keys_objects, dim3((unsigned)H.n_qtiles), dim3(OBJ_QT), 0, stream, B, dirs,
                           (uint32_t)W.n_cells, k0);
    SHM_LAUNCH_CHECK();
    radix_sort_pass_all(W, base, stream, k0, v0);
    SHM_LAUNCH_CHECK();
    launch_cell_start(W, base, k0, stream);
    const uint32_t* cs = reinterpret_cast<const uint32_t*>(base + W.cstart);
    hipLaunchKernelGGL(k_gather_rows<3>, dim3((unsigned)((W.Q + 255) / 256)), dim3(256), 0, stream, v0, dirs, W.Q,
                       reinterpret_cast<float*>(base + W.sdirs));
    if (H.n_tiles > 0) {
        const DenseTiles D = dense_tiles(base + W.dense, H.n_tiles);
        hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, stream, D.count, 0u);
        hipLaunchKernelGGL(k_tile_dense_objects, dim3((unsigned)((H.n_tiles + 3) / 4)), dim3(256), 0, stream, B,
                           H.n_tiles, (const uint32_t*)cs, D, reinterpret_cast<TileRec*>(base + W.geo));
    }
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

int launch_backward_objects(const BwdObjectsHost& H, int dtype, const void* lut, const float* dirs, const float* gout,
                            float* grad_lut, float* grad_dirs, void* ws, hipStream_t stream)
{
    const BwdLayout W = bwd_layout_cells(H.Q, H.n_cells, H.n_tiles);
    char* base = reinterpret_cast<char*>(ws);
    const uint32_t* cs = reinterpret_cast<const uint32_t*>(base + W.cstart);
    const uint32_t* perm = reinterpret_cast<const uint32_t*>(base + ((W.passes & 1) ? W.vals1 : W.vals0));
    const float* sdirs = reinterpret_cast<const float*>(base + W.sdirs);
    float* sgout = reinterpret_cast<float*>(base + W.sgout);
    const BwdObjects B{H.objs, H.cell_base, H.tile_base, H.qtile_base, H.tile_obj, H.qtile_obj, H.n_obj};
    if (grad_lut && H.n_tiles > 0) {
        if (W.Q == 0) {  // no queries: the sort wrote nothing; every object's gradient is zero
            hipLaunchKernelGGL(k_bwd_fused_objects, dim3((unsigned)H.n_tiles), dim3(BWD_THREADS), 0, stream, B,
                               (const TileRec*)nullptr, (int64_t)0, (const float*)nullptr, (const float*)nullptr,
                               (const uint32_t*)nullptr, (const uint32_t*)nullptr, grad_lut);
        } else {
            const DenseTiles D = dense_tiles(base + W.dense, H.n_tiles);
            hipLaunchKernelGGL(k_gather_rows<4>, dim3((unsigned)((W.Q + 255) / 256)), dim3(256), 0, stream, perm, gout,
                               W.Q, sgout);
            const TileRec* recs = reinterpret_cast<const TileRec*>(base + W.geo);
            hipLaunchKernelGGL(k_bwd_fused_objects, dim3((unsigned)H.n_tiles), dim3(BWD_THREADS), 0, stream, B, recs,
                               W.Q, sdirs, (const float*)sgout, perm, cs, grad_lut);
            // the plan read the dense-tile count back after its sort
            if (H.n_dense > 0)
                hipLaunchKernelGGL(k_bwd_fused_objects_dense,
                                   dim3((unsigned)std::min<int64_t>(H.n_dense, 8ll * device_cu_count())),
                                   dim3(BWD_DENSE_THREADS), 0, stream, recs, W.Q, sdirs, (const float*)sgout, perm, cs,
                                   (const uint32_t*)D.count, (const uint32_t*)D.list, grad_lut);
        }
        SHM_LAUNCH_CHECK();
    }
    if (grad_dirs && H.n_qtiles > 0) {
        if (dtype == SHM_F16)
            hipLaunchKernelGGL((k_bwd_dirs_objects<true>), dim3((unsigned)H.n_qtiles), dim3(OBJ_QT), 0, stream, B, lut,
                               dirs, gout, grad_dirs);
        else
            hipLaunchKernelGGL((k_bwd_dirs_objects<false>), dim3((unsigned)H.n_qtiles), dim3(OBJ_QT), 0, stream, B, lut,
                               dirs, gout, grad_dirs);
        SHM_LAUNCH_CHECK();
    }
    return SHM_OK;
}

const uint32_t* backward_dense_count(int N, int64_t n_obj, int64_t q_per_obj, const void* ws)
{
    return reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(ws) + bwd_layout(N, n_obj, q_per_obj).dense);
}

int launch_backward(const float* lut, int N, int64_t n_obj, const float* dirs, int64_t q_per_obj, const float* gout,
                    float* grad_lut, float* grad_dirs, void* ws, bool skip_dense, hipStream_t stream)
{
    const BwdLayout W = bwd_layout(N, n_obj, q_per_obj);
    char* base = reinterpret_cast<char*>(ws);
    const uint32_t* cs = reinterpret_cast<const uint32_t*>(base + W.cstart);
    // after an odd number of passes the sorted pairs sit in the second buffers
    const uint32_t* perm = reinterpret_cast<const uint32_t*>(base + ((W.passes & 1) ? W.vals1 : W.vals0));
    if (!grad_lut && !grad_dirs) return SHM_OK;
    if (W.Q == 0) {  // no queries: the sort wrote nothing, the gradient is zero
        if (grad_lut) {
            const int64_t n = n_obj * 6ll * (N + 2) * (N + 2);
            if (n > 0) hipLaunchKernelGGL(k_zero_f4, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                                          reinterpret_cast<float4*>(grad_lut), n);
            SHM_LAUNCH_CHECK();
        }
        return SHM_OK;
    }
    const int tpf = (N + 2 + BT - 1) / BT;
    const int64_t tiles = n_obj * 6ll * tpf * tpf;
    const int64_t dblocks = (W.Q + DIRS_THREADS - 1) / DIRS_THREADS;
    if (tiles + dblocks > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "backward: too many workgroups for one launch");
    // the LUT gradient (sorted tiles) and the direction gradients (query
    // order) are separate launches: computing the direction gradient inside
    // the tiles, interleaving both kinds of workgroup in one launch, or
    // running the two on concurrent streams all measured the same or slower
    // (the two compete for the same units: the total work sets the time)
    if (grad_lut) {
        const DenseTiles D = dense_tiles(base + W.dense, W.n_tiles);
        // skip_dense: the sparse kernel sums every tile itself (any number of
        // queries per cell is correct there, only slower)
        hipLaunchKernelGGL((k_bwd_fused<false>), dim3((unsigned)tiles), dim3(BWD_THREADS), 0, stream, lut, N,
                           texel_elems(N), W.Q, dirs, gout, perm, cs, tpf,
                           skip_dense ? nullptr : (const uint8_t*)D.flag, grad_lut, FitArgs{});
        if (!skip_dense)
            hipLaunchKernelGGL((k_bwd_fused_dense<false>), dim3((unsigned)dense_grid(tiles)), dim3(BWD_DENSE_THREADS), 0,
                               stream, lut, N, texel_elems(N), W.Q, dirs, gout, perm, cs, tpf,
                               (const uint32_t*)D.count, (const uint32_t*)D.list, grad_lut, FitArgs{});
        SHM_LAUNCH_CHECK();
    }
    if (grad_dirs) {
        hipLaunchKernelGGL(k_bwd_dirs, dim3((unsigned)dblocks), dim3(DIRS_THREADS), 0, stream, lut, N, texel_elems(N),
                           W.Q, obj_magic(q_per_obj), dirs, gout, grad_dirs);
        SHM_LAUNCH_CHECK();
    }
    return SHM_OK;
}

int launch_fit_step(const float* lut_in, float* lut_out, float* m, float* v, int N, const float* dirs, const float* tr,
                    const float* tn, int64_t Q, float w_value, int64_t step, float lr_value, float lr_deriv, float b1,
                    float b2, float eps, void* ws, bool skip_dense, hipStream_t stream)
{
    const BwdLayout W = bwd_layout(N, 1, Q);
    char* base = reinterpret_cast<char*>(ws);
    const uint32_t* cs = reinterpret_cast<const uint32_t*>(base + W.cstart);
    const uint32_t* perm = reinterpret_cast<const uint32_t*>(base + ((W.passes & 1) ? W.vals1 : W.vals0));
    const int tpf = (N + 2 + BT - 1) / BT;
    const int64_t tiles = 6ll * tpf * tpf;
    FitArgs fa;
    fa.tr = tr;
    fa.tn = tn;
    fa.w_value = w_value;
    fa.inv_q = Q > 0 ? (float)(1.0 / (double)Q) : 0.0f;
    fa.lut_out = reinterpret_cast<float4*>(lut_out);
    fa.m = reinterpret_cast<float4*>(m);
    fa.v = reinterpret_cast<float4*>(v);
    fa.k = adam_consts(step, lr_value, lr_deriv, b1, b2, eps);
    // with no queries the sort wrote nothing: every tile is sparse
    const DenseTiles D = dense_tiles(base + W.dense, W.n_tiles);
    hipLaunchKernelGGL((k_bwd_fused<true>), dim3((unsigned)tiles), dim3(BWD_THREADS), 0, stream, lut_in, N,
                       texel_elems(N), Q, dirs, (const float*)nullptr, perm, cs, tpf,
                       Q > 0 && !skip_dense ? (const uint8_t*)D.flag : nullptr, (float*)nullptr, fa);
    if (Q > 0 && !skip_dense)
        hipLaunchKernelGGL((k_bwd_fused_dense<true>), dim3((unsigned)dense_grid(tiles)), dim3(BWD_DENSE_THREADS), 0, stream,
                           lut_in, N, texel_elems(N), Q, dirs, (const float*)nullptr, perm, cs, tpf,
                           (const uint32_t*)D.count, (const uint32_t*)D.list, (float*)nullptr, fa);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

}  // namespace shm
