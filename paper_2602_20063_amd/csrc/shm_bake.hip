// LUT bake (Sec. 3.3, Alg. 1).
//
// Analytic SH mode: the bake of n_obj glyphs is the contraction
//     LUT[o][texel*4 + ch] = sum_k coeffs[o][k] * B[k][texel*4 + ch]
// with B the basis table holding, at every padded texel (gutter included),
// (Y_k, h dY_k/du, h dY_k/dv, h^2 d2Y_k/dudv).  The table is built by
// k_sh_basis with the chain rule through the chart map
//     w(u,v) = w~ / |w~|,  w~ = M + (2u-1) S + (2v-1) T
//     Y_u  = gradP . w_u,   Y_v = gradP . w_v,
//     Y_uv = w_u^T HessP w_v + gradP . w_uv,
// where P is the Cartesian polynomial form of Y_lm,
//     P_l0 = Qn_l^0(z),  P_{l,+-m} = sqrt2 Qn_l^m(z) {Re, Im}(x + i y)^m,
// Qn_l^m the normalised associated Legendre "polynomial part"
// (K_lm d^m P_l / dz^m), so gradients and Hessians are exact polynomials.
// The table is built in FP64 and stored in FP32; the contraction runs on the
// matrix cores (v_mfma_f32_16x16x4f32, FP32 operands and accumulation).
//
// The l = 0 term is left out of the table and the contraction and added
// once, in the epilogue: Y_00 is a constant with zero derivatives, so it only
// shifts the value channel, by c_00 Y_00 (rounded once from FP64).  The table
// row kt holds basis function k = kt + 1, and the contraction runs over
// K - 1 terms.  Its value is the
// bulk of R (about 1 for a glyph), and summing it first would make every
// later FP32 addition round at the scale of R rather than at the scale of
// the varying part; the derivatives of the reconstruction difference
// neighbouring texels' values (about 1.5 N times their rounding), so that
// rounding is what the gradient sees.
//
// General mode: central differences on samples taken on the padded grid
// plus a one-texel margin.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <mutex>

#include "shm_device.hpp"
#include "shm_internal.hpp"

namespace shm {

// face frame: M (major axis), S, T (sc, tc axes) of the hardware cube map
__device__ __forceinline__ void face_frame(int f, float M[3], float S[3], float T[3])
{
    for (int k = 0; k < 3; ++k) M[k] = S[k] = T[k] = 0.0f;
    switch (f) {
    case 0: M[0] = 1; S[2] = -1; T[1] = -1; break;
    case 1: M[0] = -1; S[2] = 1; T[1] = -1; break;
    case 2: M[1] = 1; S[0] = 1; T[2] = 1; break;
    case 3: M[1] = -1; S[0] = 1; T[2] = -1; break;
    case 4: M[2] = 1; S[0] = 1; T[1] = -1; break;
    default: M[2] = -1; S[0] = -1; T[1] = -1; break;
    }
}

__device__ __forceinline__ int64_t basis_index(int k, int64_t col, int Kp, int64_t rows_pad, int frag)
{
    if (!frag) return (int64_t)k * rows_pad + col;
    const int64_t t = col >> 5;
    const int c = (int)(col & 31);
    const int lane = (k & 3) * 16 + (c & 15);
    const int v = 2 * (k >> 2) + (c >> 4);  // fragment value b[j][s], v = 2 s + j
    const int G = ((Kp >> 2) + 1) >> 1;      // float4 groups per lane and tile
    return ((t * G + (v >> 2)) * 64 + lane) * 4 + (v & 3);
}

// ---------------------------------------------------------------------------
// Basis table.  One lane per padded texel; writes Bt[k-1][row] for
// k = 1 .. K-1, row = texel*4+ch (k-major so the MFMA B operand loads are
// coalesced), ld = rows_pad.
// ---------------------------------------------------------------------------
// Layouts of the table: k-major Bt[k][col] (ld = rows_pad), or, for the
// register-resident contraction, MFMA fragment order: the B fragment value
// b[j][s] of lane l for column tile t (col = 32 t + 16 j + l % 16,
// k = 4 s + l / 16) is value v = 2 s + j of the lane, and the lane's values
// sit in float4 groups Bf[t][v / 4][l][v % 4]: one tile is ceil(KS / 2)
// float4 loads per lane (KS = K / 4 steps).
template <typename Real>
__global__ void k_sh_basis(int L, int N, int Kp, int64_t rows_pad, int frag, float* __restrict__ Bt)
{
    const int P = N + 2;
    const int ntex = 6 * P * P;
    const int tex = blockIdx.x * blockDim.x + threadIdx.x;
    if (tex >= ntex) return;
    const int face = tex / (P * P);
    const int rem = tex - face * P * P;
    const int q = rem / P, p = rem - q * P;
    float Mf[3], Sf[3], Tf[3];
    face_frame(face, Mf, Sf, Tf);
    const Real invN = Real(1) / Real(N);
    const Real A = Real(2) * ((Real)p - Real(0.5)) * invN - Real(1);
    const Real B = Real(2) * ((Real)q - Real(0.5)) * invN - Real(1);
    Real w[3], wu[3], wv[3], wuv[3];
    Real rho2 = 0;
    for (int k = 0; k < 3; ++k) {
        w[k] = (Real)Mf[k] + A * (Real)Sf[k] + B * (Real)Tf[k];
        rho2 += w[k] * w[k];
    }
    const Real rho = sqrt(rho2), irho = Real(1) / rho;
    for (int k = 0; k < 3; ++k) w[k] *= irho;
    const Real wS = A * irho, wT = B * irho;  // w . S, w . T
    for (int k = 0; k < 3; ++k) {
        wu[k] = Real(2) * irho * ((Real)Sf[k] - wS * w[k]);
        wv[k] = Real(2) * irho * ((Real)Tf[k] - wT * w[k]);
        wuv[k] = Real(4) * irho * irho * (Real(3) * wS * wT * w[k] - wT * (Real)Sf[k] - wS * (Real)Tf[k]);
    }
    const Real x = w[0], y = w[1], z = w[2];
    const Real sN = invN, sN2 = invN * invN;
    const int64_t row = (int64_t)tex * 4;
    auto emit = [&](int k, Real val, const Real g[3], const Real H[6]) {
        // H = (xx, xy, xz, yy, yz, zz)
        const Real Yu = g[0] * wu[0] + g[1] * wu[1] + g[2] * wu[2];
        const Real Yv = g[0] * wv[0] + g[1] * wv[1] + g[2] * wv[2];
        const Real Hv0 = H[0] * wv[0] + H[1] * wv[1] + H[2] * wv[2];
        const Real Hv1 = H[1] * wv[0] + H[3] * wv[1] + H[4] * wv[2];
        const Real Hv2 = H[2] * wv[0] + H[4] * wv[1] + H[5] * wv[2];
        const Real Yuv = wu[0] * Hv0 + wu[1] * Hv1 + wu[2] * Hv2 + g[0] * wuv[0] + g[1] * wuv[1] + g[2] * wuv[2];
        const float v4[4] = {(float)val, (float)(Yu * sN), (float)(Yv * sN), (float)(Yuv * sN2)};
        if (k == 0) return;  // the constant l = 0 term is added by the contraction's epilogue
        for (int ch = 0; ch < 4; ++ch) Bt[basis_index(k - 1, row + ch, Kp, rows_pad, frag)] = v4[ch];
    };
    const Real SQ2 = sqrt(Real(2));
    // complex powers (x + i y)^m = A_m + i B_m, sliding window m-2..m
    Real Am2 = 0, Bm2 = 0, Am1 = 0, Bm1 = 0, Am = 1, Bm = 0;
    Real diag = Real(0.28209479177387814347);  // Qn_0^0 = 1/sqrt(4 pi)
    for (int m = 0; m <= L; ++m) {
        if (m > 0) {
            Am2 = Am1; Bm2 = Bm1;
            Am1 = Am; Bm1 = Bm;
            Am = Am1 * x - Bm1 * y;
            Bm = Am1 * y + Bm1 * x;
            diag *= sqrt(Real(2 * m + 1) / Real(2 * m));
        }
        // seeds of columns m, m+1, m+2 (diagonal values)
        const Real d0 = diag;
        const Real d1 = d0 * sqrt(Real(2 * m + 3) / Real(2 * m + 2));
        const Real d2 = d1 * sqrt(Real(2 * m + 5) / Real(2 * m + 4));
        Real c0p1 = 0, c0p2 = 0, c1p1 = 0, c1p2 = 0, c2p1 = 0, c2p2 = 0;
        for (int l = m; l <= L; ++l) {
            // column mc at order l: 0 below the diagonal, seed on it, recurrence above
            auto step = [&](int mc, Real seed, Real& p1, Real& p2) -> Real {
                Real v;
                if (l < mc) v = 0;
                else if (l == mc) v = seed;
                else {
                    const Real ll = (Real)l, mm = (Real)mc;
                    const Real a = sqrt((Real(4) * ll * ll - Real(1)) / (ll * ll - mm * mm));
                    const Real b = sqrt((((ll - 1) * (ll - 1)) - mm * mm) * (Real(2) * ll + Real(1)) /
                                        ((Real(2) * ll - Real(3)) * (ll * ll - mm * mm)));
                    v = a * z * p1 - b * p2;
                }
                p2 = p1;
                p1 = v;
                return v;
            };
            const Real q0 = step(m, d0, c0p1, c0p2);
            const Real q1 = step(m + 1, d1, c1p1, c1p2);
            const Real q2 = step(m + 2, d2, c2p1, c2p2);
            const Real f1 = sqrt(Real((l + m + 1) * (l - m)));
            const Real f2 = (l - m - 1 >= 0) ? f1 * sqrt(Real((l + m + 2) * (l - m - 1))) : Real(0);
            const Real dq = f1 * q1, d2q = f2 * q2;  // dQn/dz, d2Qn/dz2
            if (m == 0) {
                const Real g[3] = {0, 0, dq};
                const Real H[6] = {0, 0, 0, 0, 0, d2q};
                emit(l * l + l, q0, g, H);
            } else {
                const Real mm1 = (Real)(m * (m - 1));
                const Real mr = (Real)m;
                {   // +m: Re
                    const Real g[3] = {SQ2 * q0 * mr * Am1, -SQ2 * q0 * mr * Bm1, SQ2 * dq * Am};
                    const Real H[6] = {SQ2 * q0 * mm1 * Am2, -SQ2 * q0 * mm1 * Bm2, SQ2 * dq * mr * Am1,
                                       -SQ2 * q0 * mm1 * Am2, -SQ2 * dq * mr * Bm1, SQ2 * d2q * Am};
                    emit(l * l + l + m, SQ2 * q0 * Am, g, H);
                }
                {   // -m: Im
                    const Real g[3] = {SQ2 * q0 * mr * Bm1, SQ2 * q0 * mr * Am1, SQ2 * dq * Bm};
                    const Real H[6] = {SQ2 * q0 * mm1 * Bm2, SQ2 * q0 * mm1 * Am2, SQ2 * dq * mr * Bm1,
                                       -SQ2 * q0 * mm1 * Bm2, SQ2 * dq * mr * Am1, SQ2 * d2q * Bm};
                    emit(l * l + l - m, SQ2 * q0 * Bm, g, H);
                }
            }
        }
    }
    // zero padding rows (table rows K-1 .. Kp-1)
    for (int k = (L + 1) * (L + 1) - 1; k < Kp; ++k)
        for (int ch = 0; ch < 4; ++ch) Bt[basis_index(k, row + ch, Kp, rows_pad, frag)] = 0.0f;
}

// zero the padding columns rows .. rows_pad-1 of every k
__global__ void k_zero_cols(float* __restrict__ Bt, int Kp, int64_t rows, int64_t rows_pad, int frag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = rows_pad - rows;
    if (i >= w * Kp) return;
    const int64_t k = i / w, c = i - k * w;
    Bt[basis_index((int)k, rows + c, Kp, rows_pad, frag)] = 0.0f;
}

// ---------------------------------------------------------------------------
// Contraction on the matrix cores.  D[o][row] = sum_{k>=1} C[o][k] Bt[k-1][row].
// Block: 256 lanes (4 waves, 2 x 2), tile 64 objects x 128 rows; each wave
// 32 x 64 = 2 x 4 MFMA 16x16 tiles.  K is staged through LDS in chunks.
// v_mfma_f32_16x16x4f32 operand layout (lane l): A[m = l%16][k = l/16],
// B[k = l/16][n = l%16], D[m = 4*(l/16) + i][n = l%16], i = 0..3.
// ---------------------------------------------------------------------------
constexpr int GB_M = 64, GB_N = 128, GB_KC = 96;

// c_00 Y_00, Y_00 = 1 / sqrt(4 pi), formed in FP64 and rounded once
__device__ __forceinline__ float y00_term(float c00)
{
    return (float)((double)c00 * 0.28209479177387814347);
}
constexpr int GB_LDA = GB_M + 1, GB_LDB = GB_N + 16;

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <bool F16OUT>
__global__ __launch_bounds__(256) void k_bake_gemm(const float* __restrict__ C, int K, int64_t n_obj,
                                                   const float* __restrict__ Bt, int Kp, int64_t rows,
                                                   int64_t rows_pad, void* __restrict__ lut)
{
    __shared__ float As[GB_KC * GB_LDA];
    __shared__ float Bs[GB_KC * GB_LDB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;  // wave position in the 2 x 2 grid
    const int64_t o0 = (int64_t)blockIdx.y * GB_M;
    const int64_t r0 = (int64_t)blockIdx.x * GB_N;
    floatx4 acc[2][4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < Kp; kc += GB_KC) {
        const int kn = (Kp - kc) < GB_KC ? (Kp - kc) : GB_KC;  // multiple of 4
        // stage A: As[k][m] = C[o0+m][kc+k+1] (table row kc+k is term kc+k+1; zero outside)
        for (int i = tid; i < GB_M * kn; i += 256) {
            const int m = i / kn, k = i - m * kn;
            const int64_t o = o0 + m;
            const int kk = kc + k + 1;
            As[k * GB_LDA + m] = (o < n_obj && kk < K) ? C[o * K + kk] : 0.0f;
        }
        // stage B: Bs[k][n] = Bt[kc+k][r0+n]  (rows_pad covers the tile)
        for (int i = tid; i < GB_N * kn; i += 256) {
            const int k = i / GB_N, n = i - k * GB_N;
            Bs[k * GB_LDB + n] = Bt[(int64_t)(kc + k) * rows_pad + r0 + n];
        }
        __syncthreads();
        for (int k = 0; k < kn; k += 4) {
            const int kr = k + (lane >> 4);
            float a[2], b[4];
            for (int i = 0; i < 2; ++i) a[i] = As[kr * GB_LDA + wm * 32 + i * 16 + (lane & 15)];
            for (int j = 0; j < 4; ++j) b[j] = Bs[kr * GB_LDB + wn * 64 + j * 16 + (lane & 15)];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // epilogue: D[m][n] -> lut[o0 + m][r0 + n]
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 4; ++j) {
            const int64_t col = r0 + wn * 64 + j * 16 + (lane & 15);
            if (col >= rows) continue;
            for (int e = 0; e < 4; ++e) {
                const int64_t o = o0 + wm * 32 + i * 16 + 4 * (lane >> 4) + e;
                if (o >= n_obj) continue;
                // value channel (col % 4 == 0): add the l = 0 term
                const float v = (col & 3) == 0 ? acc[i][j][e] + y00_term(C[o * K]) : acc[i][j][e];
                if constexpr (F16OUT)
                    reinterpret_cast<__half*>(lut)[o * rows + col] = __float2half(v);
                else
                    reinterpret_cast<float*>(lut)[o * rows + col] = v;
            }
        }
}

// ---------------------------------------------------------------------------
// Register-resident contraction for K <= 4 * G2_KS (SH order <= 8).
// Work split: workgroup b runs on XCD b % 8 (round-robin dispatch), and XCD x
// owns column chunk x of the basis table, so that chunk (~1/8 of the table)
// stays in the XCD's L2.  Each wave owns 32 objects at a time: their
// coefficients sit in registers as MFMA A fragments for the whole K; it then
// walks the column tiles (32 columns) of its chunk, loading the B fragments
// of the next tile while the 4 x KS MFMAs of the current one run, and
// stores a 32 x 32 output tile per step, staged through the wave's own LDS
// buffer so that it leaves as whole 128 B rows.  Each tile's staging and
// stores are threaded through the next tile's MFMAs (which run
// asynchronously), so the matrix pipe does not wait for them.  No workgroup
// barriers.
// ---------------------------------------------------------------------------
constexpr int G2_KS = 20;  // K steps of 4 held in registers (K - 1 <= 80)

// Compile-time scheduling knobs of the register-resident contraction (every
// setting gives the same bits):
//   SHM_G2_MODE       0: scheduling barriers between the MFMA groups and the
//                     epilogue parts threaded through them; 1: no barriers
//                     (the compiler's order); 2: as 0, and the wave raises
//                     its priority while it issues an MFMA group
#ifndef SHM_G2_MODE
#define SHM_G2_MODE 0
#endif

__device__ __forceinline__ void g2_sep()
{
#if SHM_G2_MODE != 1
    __builtin_amdgcn_sched_barrier(0);
#endif
}

// One wave's output tile goes through LDS so that it leaves as whole rows:
// the MFMA D layout gives each lane 16 values in 4 rows of 16-column
// segments; stored directly that is 64 B pieces of four rows per
// instruction, which HBM absorbs at ~60% of the rate of full rows.  Rows are
// padded to 36 floats (16-byte aligned, banks shifted by 4 per row).
constexpr int G2_LDS_STRIDE = 36;
constexpr int G2_LDS_WAVE = 32 * G2_LDS_STRIDE;  // floats per wave

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// MFMAs of K steps [S0, S1) of one 32 x 32 output tile: four independent
// accumulator chains (2 object blocks x 2 column blocks of 16).
template <int KS, int S0, int S1>
__device__ __forceinline__ void g2_mma(const float (&a)[2][KS], const float (&b)[2][KS], floatx4 (&acc)[2][2])
{
#if SHM_G2_MODE == 2
    __builtin_amdgcn_s_setprio(1);
#endif
#pragma unroll
    for (int s = S0; s < S1; ++s)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
#if SHM_G2_MODE == 2
    __builtin_amdgcn_s_setprio(0);
#endif
}

// Epilogue, part 1: D[m][n] with m = 16 i + 4 lk + e (object), n = 16 j + lm
// (column) into the wave's LDS buffer, once the previous tile's rows have
// been read out.
__device__ __forceinline__ void g2_stage(const floatx4 (&acc)[2][2], float* __restrict__ stage, int lane)
{
    const int lm = lane & 15, lk = lane >> 4;
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) stage[(16 * i + 4 * lk + e) * G2_LDS_STRIDE + 16 * j + lm] = acc[i][j][e];
}

// Epilogue, part 2: row r = lane / 8 + 8 q, columns 4 (lane % 8) .. + 3 read
// back from LDS ...
__device__ __forceinline__ void g2_unstage(const float* __restrict__ stage, int lane, float4 (&v)[4])
{
    wave_lds_sync();
    const int cg = 4 * (lane & 7);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = *reinterpret_cast<const float4*>(stage + ((lane >> 3) + 8 * q) * G2_LDS_STRIDE + cg);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// ... and part 3: stored as whole 128 B rows; rows is a multiple of 4, so a
// group of four columns is wholly inside or outside the table
// cst[q] is the l = 0 term of object row q, added to the value channel (the
// first of each group of four columns: a texel's channels).  The stores are
// buffer stores over the wave's own object rows: a store outside the table
// (an object row past n_obj, columns past rows) gets an offset past the
// buffer's end, which the hardware drops.  No branch guards a store, so the
// compiler's count of memory operations in flight stays exact and the loop
// does not wait for its stores to finish.
template <bool F16OUT>
__device__ __forceinline__ void g2_store(float4 (&v)[4], const float (&cst)[4], int64_t o0, int64_t n_obj,
                                         int64_t col0, int64_t rows, int lane, void* __restrict__ lut)
{
    constexpr int ES = F16OUT ? 2 : 4;  // bytes per output element
    const int64_t col = col0 + 4 * (lane & 7);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q].x += cst[q];
    // an empty statement that takes every value: the LDS reads stay where
    // they were issued instead of sinking into the stores below
#pragma unroll
    for (int q = 0; q < 4; ++q) asm volatile("" : : "v"(v[q].x), "v"(v[q].y), "v"(v[q].z), "v"(v[q].w));
    // the wave's window: object rows o0 .. o0 + 31 (32 x rows x 4 B < 2^32
    // for rows <= 6 (SHM_MAX_N + 2)^2 4)
    const int64_t n_here = (n_obj - o0) < 32 ? (n_obj - o0) : 32;
    char* wbase = reinterpret_cast<char*>(lut) + o0 * rows * ES;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(wbase, (short)0, (int)(uint32_t)(n_here * rows * ES), 0x00020000);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t ol = (lane >> 3) + 8 * q;  // object row in the window
        const bool ok = ol < n_here && col < rows;
        const uint32_t off = ok ? (uint32_t)((ol * rows + col) * ES) : 0xFFFFFFF0u;
        // non-temporal: the output lines are written once and need not
        // displace the basis fragments the XCD's waves share in L2
        if constexpr (F16OUT) {
            const __half2 h0 = __floats2half2_rn(v[q].x, v[q].y), h1 = __floats2half2_rn(v[q].z, v[q].w);
            u32x2 w;
            w.x = *reinterpret_cast<const unsigned int*>(&h0);
            w.y = *reinterpret_cast<const unsigned int*>(&h1);
            __builtin_amdgcn_raw_buffer_store_b64(w, rs, off, 0, 2);
        } else {
            const u32x4 w = {__float_as_uint(v[q].x), __float_as_uint(v[q].y), __float_as_uint(v[q].z),
                             __float_as_uint(v[q].w)};
            __builtin_amdgcn_raw_buffer_store_b128(w, rs, off, 0, 2);
        }
    }
}

// One tile's MFMAs (into acc) with the epilogue of the previous tile (prev,
// column col_prev) threaded through them: the MFMAs run asynchronously, so
// the LDS writes, reads and stores issued between them keep the matrix pipe
// busy instead of following it.  The scheduling barriers keep that order.
template <bool F16OUT, int KS>
__device__ __forceinline__ void g2_tile_overlap(const float (&a)[2][KS], const float (&b)[2][KS], floatx4 (&acc)[2][2],
                                                const floatx4 (&prev)[2][2], float* __restrict__ stage,
                                                const float (&cst)[4], int64_t o0, int64_t n_obj, int64_t col_prev,
                                                int64_t rows, int lane, void* __restrict__ lut)
{
    constexpr int S1 = KS / 4, S2 = KS / 2, S3 = (3 * KS) / 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    g2_mma<KS, 0, S1>(a, b, acc);
    g2_sep();
    g2_stage(prev, stage, lane);
    g2_sep();
    g2_mma<KS, S1, S2>(a, b, acc);
    g2_sep();
    float4 v[4];
    g2_unstage(stage, lane, v);
    g2_sep();
    g2_mma<KS, S2, S3>(a, b, acc);
    g2_sep();
    g2_store<F16OUT>(v, cst, o0, n_obj, col_prev, rows, lane, lut);
    g2_sep();
    g2_mma<KS, S3, KS>(a, b, acc);
}

// The last tile's epilogue on its own.
template <bool F16OUT>
__device__ __forceinline__ void g2_flush(const floatx4 (&acc)[2][2], float* __restrict__ stage, const float (&cst)[4],
                                         int64_t o0, int64_t n_obj, int64_t col0, int64_t rows, int lane,
                                         void* __restrict__ lut)
{
    g2_stage(acc, stage, lane);
    float4 v[4];
    g2_unstage(stage, lane, v);
    g2_store<F16OUT>(v, cst, o0, n_obj, col0, rows, lane, lut);
}

// B fragments of column tile t from the fragment-ordered table: ceil(KS/2)
// float4 loads per lane (few enough that two tiles in flight stay within the
// hardware's count of outstanding loads), all offsets immediate from one base.
template <int KS>
__device__ __forceinline__ void g2_load_b(const float* __restrict__ Bf, int64_t t, int lane, float (&b)[2][KS])
{
    constexpr int G = (KS + 1) / 2;
    const float4* base = reinterpret_cast<const float4*>(Bf) + t * (int64_t)G * 64 + lane;
    float4 q[G];
#pragma unroll
    for (int g = 0; g < G; ++g) q[g] = base[g * 64];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int v = 2 * s + j;
            const float4 w = q[v >> 2];
            b[j][s] = (v & 3) == 0 ? w.x : (v & 3) == 1 ? w.y : (v & 3) == 2 ? w.z : w.w;
        }
}

template <bool F16OUT, int KS>
__global__ __launch_bounds__(256, 2) void k_bake_gemm2(const float* __restrict__ C, int K, int64_t n_obj,
                                                       const float* __restrict__ Bt, int64_t rows,
                                                       int64_t rows_pad, void* __restrict__ lut, int waves_per_xcd,
                                                       int n_sub)
{
    __shared__ __attribute__((aligned(16))) float stage_all[4 * G2_LDS_WAVE];
    float* stage = stage_all + (threadIdx.x >> 6) * G2_LDS_WAVE;
    // XCD x owns column chunk x; the chunk is cut into n_sub sub-chunks and
    // the work units (object group, sub-chunk) are dealt to the XCD's waves
    const int lane = threadIdx.x & 63;
    const int xcd = blockIdx.x & 7;
    // wave-uniform (read from lane 0) so that the loops below are scalar: a
    // loop the compiler takes as divergent gets exec-mask branches and waits
    // for all outstanding memory operations at every join
    const int wave_in_xcd = __builtin_amdgcn_readfirstlane((int)(blockIdx.x >> 3) * 4 + (int)(threadIdx.x >> 6));
    const int64_t ntiles = rows_pad / 32;  // column tiles of 32
    const int64_t per_chunk = (ntiles + 7) / 8;
    const int64_t c_begin = xcd * per_chunk;
    const int64_t c_end = (c_begin + per_chunk) < ntiles ? (c_begin + per_chunk) : ntiles;
    const int64_t per_sub = (per_chunk + n_sub - 1) / n_sub;
    const int64_t n_og = (n_obj + 31) / 32;
    const int lm = lane & 15, lk = lane >> 4;
    for (int64_t u = wave_in_xcd; u < n_og * n_sub; u += waves_per_xcd) {
        const int64_t og = u / n_sub, sub = u - og * n_sub;
        const int64_t t_begin = c_begin + sub * per_sub;
        const int64_t t_end = (t_begin + per_sub) < c_end ? (t_begin + per_sub) : c_end;
        if (t_begin >= t_end) continue;
        const int64_t o0 = og * 32;
        // loads are unconditional (clamped addresses, then a select), so the
        // compiler's wait counts stay exact and the prefetch below overlaps
        float a[2][KS];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int64_t o = o0 + 16 * i + lm;
            const int64_t oc = o < n_obj ? o : n_obj - 1;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                // table row 4 s + lk holds term k = 4 s + lk + 1 (the l = 0
                // term is added in the epilogue)
                const int k = 4 * s + lk + 1;
                const float v = C[oc * K + (k < K ? k : K - 1)];
                // zero outside the table by a bit mask: a select would let the
                // compiler sink the load into a branch of its own
                const unsigned int keep = (o < n_obj && k < K) ? 0xffffffffu : 0u;
                a[i][s] = __uint_as_float(__float_as_uint(v) & keep);
            }
        }
        // l = 0 terms of the four object rows this lane stores
        float cst[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t o = o0 + (lane >> 3) + 8 * q;
            cst[q] = y00_term(C[(o < n_obj ? o : n_obj - 1) * K]);
        }
        // tile k (k = 0 .. n-1 from t_begin) uses B buffer k % 2 and
        // accumulators k % 2; a buffer reloads (two tiles ahead) once its
        // MFMAs have issued, and tile k's epilogue runs inside tile k+1's
        // MFMAs (past the last tile the last one is loaded again, unused)
        const int64_t n = t_end - t_begin;
        auto tile_at = [&](int64_t k) { return t_begin + (k < n ? k : n - 1); };
        float b0[2][KS], b1[2][KS];
        floatx4 c0[2][2], c1[2][2];
        g2_load_b<KS>(Bt, tile_at(0), lane, b0);
        g2_load_b<KS>(Bt, tile_at(1), lane, b1);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) c0[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
        g2_mma<KS, 0, KS>(a, b0, c0);
        g2_load_b<KS>(Bt, tile_at(2), lane, b0);
        for (int64_t k = 1;; k += 2) {
            if (k >= n) {
                g2_flush<F16OUT>(c0, stage, cst, o0, n_obj, tile_at(k - 1) * 32, rows, lane, lut);
                break;
            }
            g2_tile_overlap<F16OUT, KS>(a, b1, c1, c0, stage, cst, o0, n_obj, tile_at(k - 1) * 32, rows, lane, lut);
            g2_load_b<KS>(Bt, tile_at(k + 2), lane, b1);
            if (k + 1 >= n) {
                g2_flush<F16OUT>(c1, stage, cst, o0, n_obj, tile_at(k) * 32, rows, lane, lut);
                break;
            }
            g2_tile_overlap<F16OUT, KS>(a, b0, c0, c1, stage, cst, o0, n_obj, tile_at(k) * 32, rows, lane, lut);
            g2_load_b<KS>(Bt, tile_at(k + 3), lane, b0);
        }
    }
}

// table rows: the K - 1 terms l >= 1, rounded up to a multiple of 4 (at least 4)
static inline int bake_kp(int L)
{
    const int kt = (L + 1) * (L + 1) - 1;
    return kt < 4 ? 4 : (kt + 3) / 4 * 4;
}
static inline int64_t bake_rows(int N) { return texel_elems(N); }
static inline int64_t bake_rows_pad(int N) { return (bake_rows(N) + GB_N - 1) / GB_N * GB_N; }

// K-major: Kp x rows_pad; fragment order: rows_pad x 8 ceil(Kp / 8) (4 more
// K rows when Kp / 4 is odd)
size_t bake_workspace_bytes(int L, int N) { return (size_t)(bake_kp(L) + 4) * (size_t)bake_rows_pad(N) * sizeof(float); }

int launch_bake_sh(const float* coeffs, int L, int N, int64_t n_obj, int out_dtype, void* lut, void* ws,
                   hipStream_t stream)
{
    const int K = (L + 1) * (L + 1), Kp = bake_kp(L);
    const int64_t rows = bake_rows(N), rows_pad = bake_rows_pad(N);
    float* Bt = reinterpret_cast<float*>(ws);
    const int ntex = 6 * (N + 2) * (N + 2);
    const bool regs = Kp <= 4 * G2_KS;  // register-resident contraction (fragment-ordered table)
    // The table is evaluated in FP64 at every order (it is a vanishing part
    // of the bake's arithmetic) so that it adds nothing beyond its FP32
    // storage rounding: the tangential chain rule cancels the radial part of
    // the Cartesian polynomial's gradient, which grows with the SH order.
    hipLaunchKernelGGL(k_sh_basis<double>, dim3((ntex + 127) / 128), dim3(128), 0, stream, L, N, Kp, rows_pad,
                       regs ? 1 : 0, Bt);
    SHM_LAUNCH_CHECK();
    if (rows_pad > rows) {
        const int64_t n = (rows_pad - rows) * Kp;
        hipLaunchKernelGGL(k_zero_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, Bt, Kp, rows, rows_pad,
                           regs ? 1 : 0);
        SHM_LAUNCH_CHECK();
    }
    if (regs) {
        // 8 XCDs x blocks_per_xcd workgroups of 4 waves, two workgroups per CU
        const int n_cu = device_cu_count();
        const int64_t n_og = (n_obj + 31) / 32;
        int64_t per_xcd = (int64_t)(n_cu / 8) * 2;
        if (per_xcd < 1) per_xcd = 1;
        const int waves_per_xcd = (int)per_xcd * 4;
        // enough (object group, column sub-chunk) units for every wave
        const int64_t ntiles = rows_pad / 32, per_chunk = (ntiles + 7) / 8;
        int64_t n_sub = (waves_per_xcd + n_og - 1) / n_og;
        if (n_sub > per_chunk) n_sub = per_chunk;
        if (n_sub < 1) n_sub = 1;
        const dim3 grid((unsigned)(per_xcd * 8));
        const bool f16 = out_dtype == SHM_F16;
        // the K steps are a compile-time count: loads and MFMAs are straight-line code
#define SHM_G2(KSV)                                                                                                  \
    case KSV:                                                                                                        \
        if (f16)                                                                                                     \
            hipLaunchKernelGGL((k_bake_gemm2<true, KSV>), grid, dim3(256), 0, stream, coeffs, K, n_obj, Bt, rows,     \
                               rows_pad, lut, waves_per_xcd, (int)n_sub);                                            \
        else                                                                                                         \
            hipLaunchKernelGGL((k_bake_gemm2<false, KSV>), grid, dim3(256), 0, stream, coeffs, K, n_obj, Bt, rows,    \
                               rows_pad, lut, waves_per_xcd, (int)n_sub);                                            \
        break;
        switch (Kp / 4) {  // L = 0..8: (L + 1)^2 - 1 rounded up to a multiple of 4, in steps of 4
            SHM_G2(1)
            SHM_G2(2)
            SHM_G2(4)
            SHM_G2(6)
            SHM_G2(9)
            SHM_G2(12)
            SHM_G2(16)
            SHM_G2(20)
            default:
                return fail(SHM_ERR_UNSUPPORTED, "bake: no contraction kernel for %d K steps", Kp / 4);
        }
#undef SHM_G2
        SHM_LAUNCH_CHECK();
        return SHM_OK;
    }
    const int64_t gy = (n_obj + GB_M - 1) / GB_M;
    const int64_t gx = rows_pad / GB_N;
    if (gy > 65535 * 16 || gx > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "bake: too many objects for one launch");
    // grid.y is limited; split objects into launches of <= 65535 tiles
    for (int64_t y0 = 0; y0 < gy; y0 += 65535) {
        const int64_t ny = (gy - y0) < 65535 ? (gy - y0) : 65535;
        const int64_t ob = y0 * GB_M;
        const int64_t nob = (n_obj - ob) < ny * GB_M ? (n_obj - ob) : ny * GB_M;
        const dim3 grid((unsigned)gx, (unsigned)ny);
        if (out_dtype == SHM_F16)
            hipLaunchKernelGGL(k_bake_gemm<true>, grid, dim3(256), 0, stream, coeffs + ob * K, K, nob, Bt, Kp, rows,
                               rows_pad, (void*)(reinterpret_cast<__half*>(lut) + ob * rows));
        else
            hipLaunchKernelGGL(k_bake_gemm<false>, grid, dim3(256), 0, stream, coeffs + ob * K, K, nob, Bt, Kp, rows,
                               rows_pad, (void*)(reinterpret_cast<float*>(lut) + ob * rows));
        SHM_LAUNCH_CHECK();
    }
    return SHM_OK;
}

// ---------------------------------------------------------------------------
// The bake without a caller workspace, for callers that cannot allocate: the
// basis table goes to a file-scope device array of SHM_BAKE_NOALLOC_MAX_BYTES
// (each device the library runs on holds its own copy until the process
// ends).  Host code never passes the array's name to a kernel: its device
// address is looked up once per device, with that device current, and kept.
// Every call on a device uses the same array; the table is rewritten in full
// by each call (nothing in it needs clearing), so calls that overlap on one
// device race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[SHM_BAKE_NOALLOC_MAX_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];  // device address of `scratch` per device

static int scratch_address(void** out)
{
    int dev = 0;
    SHM_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(SHM_ERR_UNSUPPORTED, "bake_noalloc: device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        SHM_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SHM_ERR_HIP, "bake_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SHM_OK;
}

int launch_bake_sh_noalloc(const float* coeffs, int L, int N, int64_t n_obj, int out_dtype, void* lut,
                           hipStream_t stream)
{
    void* ws = nullptr;
    if (int rc = scratch_address(&ws)) return rc;
    return launch_bake_sh(coeffs, L, N, n_obj, out_dtype, lut, ws, stream);
}

// ---------------------------------------------------------------------------
// General mode: sample directions and central differences.
// ---------------------------------------------------------------------------
__global__ void k_margin_dirs(int N, float* __restrict__ dirs)
{
    const int P = N + 4;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 6 * P * P) return;
    const int face = i / (P * P), rem = i - face * P * P;
    const int q = rem / P, p = rem - q * P;
    float M[3], S[3], T[3];
    face_frame(face, M, S, T);
    const float A = 2.0f * ((float)p - 1.5f) / (float)N - 1.0f;
    const float B = 2.0f * ((float)q - 1.5f) / (float)N - 1.0f;
    float w[3], n2 = 0.f;
    for (int k = 0; k < 3; ++k) { w[k] = M[k] + A * S[k] + B * T[k]; n2 += w[k] * w[k]; }
    const float in = 1.0f / sqrtf(n2);
    for (int k = 0; k < 3; ++k) dirs[(int64_t)i * 3 + k] = w[k] * in;
}

template <bool F16OUT>
__global__ void k_bake_fd(const float* __restrict__ samples, int N, int64_t n_obj, void* __restrict__ lut)
{
    const int P = N + 2, Pm = N + 4;
    const int64_t per = 6ll * P * P;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= per * n_obj) return;
    const int64_t obj = i / per;
    const int rem = (int)(i - obj * per);
    const int face = rem / (P * P), r2 = rem - face * P * P;
    const int q = r2 / P, p = r2 - q * P;
    const float* S = samples + obj * 6ll * Pm * Pm + (int64_t)face * Pm * Pm;
    const int pp = p + 1, qq = q + 1;
    auto at = [&](int a, int b) { return S[(int64_t)b * Pm + a]; };
    const float c = at(pp, qq);
    const float du = 0.5f * (at(pp + 1, qq) - at(pp - 1, qq));
    const float dv = 0.5f * (at(pp, qq + 1) - at(pp, qq - 1));
    const float duv = 0.25f * ((at(pp + 1, qq + 1) - at(pp + 1, qq - 1)) - (at(pp - 1, qq + 1) - at(pp - 1, qq - 1)));
    if constexpr (F16OUT) {
        __half* o = reinterpret_cast<__half*>(lut) + i * 4;
        o[0] = __float2half(c); o[1] = __float2half(du); o[2] = __float2half(dv); o[3] = __float2half(duv);
    } else {
        reinterpret_cast<float4*>(lut)[i] = make_float4(c, du, dv, duv);
    }
}

int launch_margin_dirs(int N, float* dirs, hipStream_t stream)
{
    const int n = 6 * (N + 4) * (N + 4);
    hipLaunchKernelGGL(k_margin_dirs, dim3((n + 255) / 256), dim3(256), 0, stream, N, dirs);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

int launch_bake_fd(const float* samples, int N, int64_t n_obj, int out_dtype, void* lut, hipStream_t stream)
{
    const int64_t n = 6ll * (N + 2) * (N + 2) * n_obj;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return fail(SHM_ERR_UNSUPPORTED, "bake_fd: too large");
    if (out_dtype == SHM_F16)
        hipLaunchKernelGGL(k_bake_fd<true>, dim3((unsigned)blocks), dim3(256), 0, stream, samples, N, n_obj, lut);
    else
        hipLaunchKernelGGL(k_bake_fd<false>, dim3((unsigned)blocks), dim3(256), 0, stream, samples, N, n_obj, lut);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

// ---------------------------------------------------------------------------
// Bernstein bound of the reconstruction (largest Bezier control point of any
// cell; with SHM_SIGNED the largest |control point|, which bounds |r|).
// 1-D Hermite (p0, m0, p1, m1) -> Bezier (p0, p0+m0/3, p1-m1/3, p1), tensor
// product over the cell.  Max-reduction through the order-preserving integer
// image of non-negative floats is exact; a negative bound clamps to 0
// (R >= 0 for a star-shaped surface).
// ---------------------------------------------------------------------------
// Largest Bezier control point of cell (i0, j0) of a face (convex hull
// bound of its bicubic patch); with absval the largest |control point|.
template <bool F16, bool CELL>
__device__ __forceinline__ float cell_bezier_max(const void* __restrict__ lut, int N, int face, int i0, int j0,
                                                 bool absval)
{
    const int P = N + 2;
    float G[4][4];  // [s-index over (p0, m0, p1, m1)][t-index likewise]
    Foot F;
    if constexpr (CELL) {  // the cell's footprint as a query decodes it
        Loc L{};
        L.face = face;
        L.i0 = i0;
        L.j0 = j0;
        F = load_foot<F16, true>(lut, N, L);
    }
    for (int dj = 0; dj < 2; ++dj)
        for (int di = 0; di < 2; ++di) {
            const int64_t t = ((int64_t)(face * P + j0 + dj) * P + i0 + di) * 4;
            float c[4];
            if constexpr (CELL) {
                const float4 v = F.c[dj * 2 + di];
                c[0] = v.x;
                c[1] = v.y;
                c[2] = v.z;
                c[3] = v.w;
            } else if constexpr (F16) {
                const __half* h = reinterpret_cast<const __half*>(lut) + t;
                for (int k = 0; k < 4; ++k) c[k] = __half2float(h[k]);
            } else {
                const float* f = reinterpret_cast<const float*>(lut) + t;
                for (int k = 0; k < 4; ++k) c[k] = f[k];
            }
            G[2 * di][2 * dj] = c[0];
            G[2 * di + 1][2 * dj] = c[1];
            G[2 * di][2 * dj + 1] = c[2];
            G[2 * di + 1][2 * dj + 1] = c[3];
        }
    float H[4][4];
    for (int b = 0; b < 4; ++b) {
        H[0][b] = G[0][b];
        H[1][b] = G[0][b] + G[1][b] / 3.0f;
        H[2][b] = G[2][b] - G[3][b] / 3.0f;
        H[3][b] = G[2][b];
    }
    float best = -__builtin_inff();
    for (int a = 0; a < 4; ++a) {
        float z0 = H[a][0], z1 = H[a][0] + H[a][1] / 3.0f, z2 = H[a][2] - H[a][3] / 3.0f, z3 = H[a][2];
        if (absval) {
            z0 = fabsf(z0);
            z1 = fabsf(z1);
            z2 = fabsf(z2);
            z3 = fabsf(z3);
        }
        best = fmaxf(best, fmaxf(fmaxf(z0, z1), fmaxf(z2, z3)));
    }
    return best;
}

template <bool F16, bool CELL>
__global__ void k_lut_rmax(const void* __restrict__ lut, int N, int absval, unsigned int* __restrict__ out_bits)
{
    const int C = N + 1;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float best = 0.0f;
    if (i < 6 * C * C) {
        const int face = i / (C * C), rem = i - face * C * C;
        const int j0 = rem / C, i0 = rem - j0 * C;
        best = fmaxf(best, cell_bezier_max<F16, CELL>(lut, N, face, i0, j0, absval != 0));
    }
    // wave reduction, then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) best = fmaxf(best, __shfl_xor(best, off));
    if ((threadIdx.x & 63) == 0) atomicMax(out_bits, __float_as_uint(best));
}

// Block bound map: face f is cut into B x B blocks of (u, v) (block bi covers
// u in [bi/B, (bi+1)/B]); map[f][bj][bi] = max(0, the largest control point
// of the cells that block can reach, widened by one cell on every side so
// that a direction located to within an ulp of a block edge is still
// covered).  One 64-lane workgroup per block: lanes stride over the cells,
// then a wave maximum.  The trace uses it to skip march samples that are
// provably outside the surface.
template <bool F16, bool CELL>
__global__ void k_bound_map(const void* __restrict__ lut, int N, int absval, int B, float* __restrict__ map)
{
    const int blk = blockIdx.x;
    const int face = blk / (B * B), rem = blk - face * B * B;
    const int bj = rem / B, bi = rem - bj * B;
    // cells i0 = floor(u N + 1/2) for u in the block, in integers
    const int i_lo = max((2 * bi * N + B) / (2 * B) - 1, 0), i_hi = min((2 * (bi + 1) * N + B) / (2 * B) + 1, N);
    const int j_lo = max((2 * bj * N + B) / (2 * B) - 1, 0), j_hi = min((2 * (bj + 1) * N + B) / (2 * B) + 1, N);
    const int wi = i_hi - i_lo + 1, n = wi * (j_hi - j_lo + 1);
    float best = 0.0f;
    for (int k = threadIdx.x; k < n; k += 64) {
        const int j0 = j_lo + k / wi, i0 = i_lo + k % wi;
        best = fmaxf(best, cell_bezier_max<F16, CELL>(lut, N, face, i0, j0, absval != 0));
    }
    for (int off = 32; off > 0; off >>= 1) best = fmaxf(best, __shfl_xor(best, off));
    if (threadIdx.x == 0) map[blk] = best;
}

__global__ void k_bits_to_float(const unsigned int* bits, float* out) { *out = __uint_as_float(*bits); }

__global__ void k_fill_u32(unsigned int* p, unsigned int v) { *p = v; }

int launch_lut_rmax(const void* lut, int dtype, int N, int flags, float* rmax_out, hipStream_t stream)
{
    unsigned int* bits = reinterpret_cast<unsigned int*>(rmax_out);  // reuse the output word
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, stream, bits, 0u);
    const int n = 6 * (N + 1) * (N + 1);
    const int absval = (flags & SHM_SIGNED) ? 1 : 0;
    const dim3 grid((n + 255) / 256), bl(256);
    if (flags & SHM_CELL_LUT) {
        if (dtype == SHM_F16) hipLaunchKernelGGL((k_lut_rmax<true, true>), grid, bl, 0, stream, lut, N, absval, bits);
        else hipLaunchKernelGGL((k_lut_rmax<false, true>), grid, bl, 0, stream, lut, N, absval, bits);
    } else {
        if (dtype == SHM_F16) hipLaunchKernelGGL((k_lut_rmax<true, false>), grid, bl, 0, stream, lut, N, absval, bits);
        else hipLaunchKernelGGL((k_lut_rmax<false, false>), grid, bl, 0, stream, lut, N, absval, bits);
    }
    hipLaunchKernelGGL(k_bits_to_float, dim3(1), dim3(1), 0, stream, bits, rmax_out);
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

int launch_bound_map(const void* lut, int dtype, int N, int flags, int blocks, float* map, hipStream_t stream)
{
    const int absval = (flags & SHM_SIGNED) ? 1 : 0;
    const dim3 grid((unsigned)(6 * blocks * blocks)), bl(64);
    if (flags & SHM_CELL_LUT) {
        if (dtype == SHM_F16) hipLaunchKernelGGL((k_bound_map<true, true>), grid, bl, 0, stream, lut, N, absval, blocks, map);
        else hipLaunchKernelGGL((k_bound_map<false, true>), grid, bl, 0, stream, lut, N, absval, blocks, map);
    } else {
        if (dtype == SHM_F16) hipLaunchKernelGGL((k_bound_map<true, false>), grid, bl, 0, stream, lut, N, absval, blocks, map);
        else hipLaunchKernelGGL((k_bound_map<false, false>), grid, bl, 0, stream, lut, N, absval, blocks, map);
    }
    SHM_LAUNCH_CHECK();
    return SHM_OK;
}

}  // namespace shm
