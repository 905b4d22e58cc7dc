// Device-side building blocks of the Spherical Hermite Map query (gfx950).
//
//   locate()      direction -> cube-map face, cell and local (s, t)   Sec. 3.2
//   load_*()      the 2x2 footprint (16 scalars) from a TEXEL or CELL LUT
//   hermite()     value and chart derivatives, Eqs. (3)-(5)
//   transport()   chart derivatives -> spherical gradient, Sec. 3.4
//
// The gradient uses the closed form of the metric-tensor solve of
// Eqs. (6)-(9): with a = sc/ma, b = tc/ma and rho = sqrt(1 + a^2 + b^2),
//   grad R = (rho / 2) [ r_u (S - a M) + r_v (T - b M) ],
// which is what Cramer's rule returns for e1 = dw/du, e2 = dw/dv on the
// face (det G = 16 / rho^6 >= 16/27 there, so the clamp never acts).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

// Cache policy of the footprint loads: each cell is touched by one query,
// so the loads can bypass the caches' retention (non-temporal).
#ifndef SHM_LUT_NT
#define SHM_LUT_NT 0
#endif

namespace shm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));

__device__ __forceinline__ float4 ld_f4(const float4* p)
{
#if SHM_LUT_NT
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
#else
    return *p;
#endif
}

__device__ __forceinline__ uint4 ld_u4(const uint4* p)
{
#if SHM_LUT_NT
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
#else
    return *p;
#endif
}

struct Loc {
    int face;     // 0..5 = +X, -X, +Y, -Y, +Z, -Z; -1 = invalid direction
    int i0, j0;   // cell: corners are padded texels (i0+{0,1}, j0+{0,1})
    float s, t;   // local coordinates in the cell
    float a, b;   // sc/ma, tc/ma in [-1, 1]
};

// Face selection on the raw components, ties X > Y > Z, sign >= 0 -> +face.
// The integer decision follows exactly: a = sc/ma, u = (a+1)*0.5,
// f = u*N + 0.5, i0 = min(floor(f), N), each step rounded to nearest (no
// contraction).  The local coordinate s is then formed to ~1 ulp of s from
// a double-float a (residual of the division by fma) instead of f - i0,
// whose error grows like ulp(N).
// FAST: the four divisions by ma use the hardware reciprocal (~1 ulp)
// instead of correctly rounded division.  s and t stay accurate to ~1 ulp
// (the residual sc - a ma is still exact), but a direction within an ulp of
// a cell boundary may be given to the neighbouring cell, whose patch agrees
// there by C1 continuity; only the ray-casting iterations use it.
// Workgroups are dispatched round-robin over the 8 XCDs; map them so that
// consecutive logical tiles share an XCD (and its L2): XCD x takes the
// contiguous range of logical ids after those of XCDs 0..x-1.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int xcd = b & 7, local = b >> 3;
    const int start = xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q;
    return start + local;
}

// Power-of-two prescale for a direction with largest component ma: 2^100
// below 2^-60 and 2^-100 above 2^60, else 1, so that the scaled ma lies in
// [2^-49, 2^40] for every finite nonzero ma (subnormal ones included) and its
// square in the normal range.  Scaling up is exact; scaling down may round
// components more than 2^24 times smaller than ma, below FP32 resolution of
// the unit vector.
__device__ __forceinline__ float dir_prescale(float ma)
{
    return ma < 0x1p-60f ? 0x1p100f : (ma > 0x1p60f ? 0x1p-100f : 1.0f);
}

// The unit vector d/|d| of a nonzero finite d of any magnitude.
__device__ __forceinline__ float3 unit_dir(float x, float y, float z)
{
#pragma clang fp contract(on)
    const float k = dir_prescale(fmaxf(fabsf(x), fmaxf(fabsf(y), fabsf(z))));
    x *= k;
    y *= k;
    z *= k;
    const float il = rsqrtf(x * x + y * y + z * z);
    return make_float3(x * il, y * il, z * il);
}

template <bool FAST>
__device__ __forceinline__ Loc locate_t(float x, float y, float z, int N)
{
#pragma clang fp contract(off)
    Loc L;
    const float ax = fabsf(x), ay = fabsf(y), az = fabsf(z);
    const bool isx = (ax >= ay) && (ax >= az);
    const bool isy = !isx && (ay >= az);
    // selects, not branches: a branch would wait for every load in flight
    const bool pos = (isx ? x : (isy ? y : z)) >= 0.0f;
    int face = (isx ? 0 : (isy ? 2 : 4)) + (pos ? 0 : 1);
    float ma = isx ? ax : (isy ? ay : az);
    float sc = isx ? (pos ? -z : z) : (isy ? x : (pos ? x : -x));
    float tc = isy ? (pos ? z : -z) : -y;
    const bool ok = isfinite(x) && isfinite(y) && isfinite(z) && (ma > 0.0f);
    if (!FAST) {
        // a major axis below 2^-64 (subnormal ones included) is scaled by
        // 2^64 first, exactly: a = sc/ma is the same correctly rounded
        // quotient, and 1/ma in the residual below cannot overflow
        const float k = ma < 0x1p-64f ? 0x1p64f : 1.0f;
        sc *= k;
        tc *= k;
        ma *= k;
    }
    const float rma = FAST ? __builtin_amdgcn_rcpf(ma) : 0.0f;
    const float a = FAST ? sc * rma : sc / ma;
    const float b = FAST ? tc * rma : tc / ma;
    const float u = (a + 1.0f) * 0.5f;
    const float v = (b + 1.0f) * 0.5f;
    const float Nf = (float)N;
    float fu = u * Nf;
    float fv = v * Nf;
    fu = fu + 0.5f;
    fv = fv + 0.5f;
    int i0 = (int)floorf(fu);
    int j0 = (int)floorf(fv);
    i0 = i0 > N ? N : (i0 < 0 ? 0 : i0);
    j0 = j0 > N ? N : (j0 < 0 ? 0 : j0);
    // s = (a + 1) N/2 + 1/2 - i0 with a = a_hi + a_lo (exact residual)
    // the residual terms only refine s, t below FP32 resolution (they are
    // ~ulp(a)): the hardware reciprocal is exact enough for them, and the
    // decisions above used the correctly rounded a, b
    const float ir = FAST ? rma : __builtin_amdgcn_rcpf(ma);
    const float a_lo = __builtin_fmaf(-a, ma, sc) * ir;
    const float b_lo = __builtin_fmaf(-b, ma, tc) * ir;
    const float halfN = 0.5f * Nf;
    const float cu = (halfN + 0.5f) - (float)i0;  // exact: half-integers below 2^23
    const float cv = (halfN + 0.5f) - (float)j0;
    L.s = __builtin_fmaf(a, halfN, cu) + a_lo * halfN;
    L.t = __builtin_fmaf(b, halfN, cv) + b_lo * halfN;
    L.a = a;
    L.b = b;
    L.i0 = i0;
    L.j0 = j0;
    L.face = ok ? face : -1;
    return L;
}

__device__ __forceinline__ Loc locate(float x, float y, float z, int N) { return locate_t<false>(x, y, z, N); }

// 16 footprint scalars: c[corner][ch], corner 0 = (i0,j0), 1 = (i0+1,j0),
// 2 = (i0,j0+1), 3 = (i0+1,j0+1); ch = (r, r_u h, r_v h, r_uv h^2).
struct Foot {
    float4 c[4];
};

__device__ __forceinline__ float4 h4_to_f4(uint2 h)
{
    const __half2 lo = *reinterpret_cast<const __half2*>(&h.x);
    const __half2 hi = *reinterpret_cast<const __half2*>(&h.y);
    const float2 a = __half22float2(lo), b = __half22float2(hi);
    return make_float4(a.x, a.y, b.x, b.y);
}

// A footprint as loaded, before any conversion: FP32 layouts load the four
// corners as they are; FP16 cells load two 16 B halves, FP16 texels four 8 B
// corners.  decode() turns it into the 16 FP32 scalars.
template <bool FP16, bool CELL>
struct FootRaw {
    float4 c[4];
};
template <>
struct FootRaw<true, true> {
    uint4 q[2];
};
template <>
struct FootRaw<true, false> {
    uint2 h[4];
};

// TEXEL layout: two rows of two texels (2 x 32 B in FP32, 2 x 16 B in FP16).
__device__ __forceinline__ FootRaw<false, false> load_raw_texel_f32(const float* __restrict__ lut, int N, const Loc& L)
{
    const int P = N + 2;
    const int64_t row0 = ((int64_t)(L.face * P + L.j0) * P + L.i0) * 4;
    const float4* p0 = reinterpret_cast<const float4*>(lut + row0);
    const float4* p1 = reinterpret_cast<const float4*>(lut + row0 + (int64_t)P * 4);
    FootRaw<false, false> R;
    R.c[0] = *(p0);
    R.c[1] = *(p0 + 1);
    R.c[2] = *(p1);
    R.c[3] = *(p1 + 1);
    return R;
}

__device__ __forceinline__ FootRaw<true, false> load_raw_texel_f16(const __half* __restrict__ lut, int N, const Loc& L)
{
    const int P = N + 2;
    const int64_t row0 = ((int64_t)(L.face * P + L.j0) * P + L.i0) * 4;
    const uint2* p0 = reinterpret_cast<const uint2*>(lut + row0);
    const uint2* p1 = reinterpret_cast<const uint2*>(lut + row0 + (int64_t)P * 4);
    FootRaw<true, false> R;
    R.h[0] = *(p0);
    R.h[1] = *(p0 + 1);
    R.h[2] = *(p1);
    R.h[3] = *(p1 + 1);
    return R;
}

// CELL layout: one contiguous, aligned block per cell.
__device__ __forceinline__ FootRaw<false, true> load_raw_cell_f32(const float* __restrict__ lut, int N, const Loc& L)
{
    const int C = N + 1;
    const int64_t cell = (int64_t)(L.face * C + L.j0) * C + L.i0;
    const float4* p = reinterpret_cast<const float4*>(lut + cell * 16);
    FootRaw<false, true> R;
    R.c[0] = ld_f4(p);
    R.c[1] = ld_f4(p + 1);
    R.c[2] = ld_f4(p + 2);
    R.c[3] = ld_f4(p + 3);
    return R;
}

__device__ __forceinline__ FootRaw<true, true> load_raw_cell_f16(const __half* __restrict__ lut, int N, const Loc& L)
{
    const int C = N + 1;
    const int64_t cell = (int64_t)(L.face * C + L.j0) * C + L.i0;
    const uint4* p = reinterpret_cast<const uint4*>(lut + cell * 16);
    FootRaw<true, true> R;
    R.q[0] = ld_u4(p);
    R.q[1] = ld_u4(p + 1);
    return R;
}

template <bool FP16, bool CELL>
__device__ __forceinline__ FootRaw<FP16, CELL> load_raw(const void* __restrict__ lut, int N, const Loc& L)
{
    if constexpr (CELL) {
        if constexpr (FP16) return load_raw_cell_f16(reinterpret_cast<const __half*>(lut), N, L);
        else return load_raw_cell_f32(reinterpret_cast<const float*>(lut), N, L);
    } else {
        if constexpr (FP16) return load_raw_texel_f16(reinterpret_cast<const __half*>(lut), N, L);
        else return load_raw_texel_f32(reinterpret_cast<const float*>(lut), N, L);
    }
}

template <bool FP16, bool CELL>
__device__ __forceinline__ Foot decode(const FootRaw<FP16, CELL>& R)
{
#pragma clang fp contract(on)
    Foot F;
    if constexpr (!FP16) {
#pragma unroll
        for (int c = 0; c < 4; ++c) F.c[c] = R.c[c];
    } else if constexpr (!CELL) {
#pragma unroll
        for (int c = 0; c < 4; ++c) F.c[c] = h4_to_f4(R.h[c]);
    } else {
        // FP16 cell encoding: corner 0 stores (r, r_u h, r_v h, r_uv h^2);
        // corners 1..3 store the value r as its difference from corner 0's
        // r.  Derivatives of the patch weigh the corner values by basis
        // functions that sum to zero, so the rounding of corner 0's r cancels
        // from them exactly and only the (small) differences are rounded:
        // the gradient keeps FP16's relative precision instead of losing a
        // factor ~N to the value's rounding.
        F.c[0] = h4_to_f4(make_uint2(R.q[0].x, R.q[0].y));
        F.c[1] = h4_to_f4(make_uint2(R.q[0].z, R.q[0].w));
        F.c[2] = h4_to_f4(make_uint2(R.q[1].x, R.q[1].y));
        F.c[3] = h4_to_f4(make_uint2(R.q[1].z, R.q[1].w));
        F.c[1].x += F.c[0].x;
        F.c[2].x += F.c[0].x;
        F.c[3].x += F.c[0].x;
    }
    return F;
}

// An empty statement that takes (and may change) a loaded footprint's
// registers: code after it cannot start before the load is issued.
__device__ __forceinline__ void pin(FootRaw<true, true>& R)
{
#pragma unroll
    for (int i = 0; i < 2; ++i) asm volatile("" : "+v"(R.q[i].x), "+v"(R.q[i].y), "+v"(R.q[i].z), "+v"(R.q[i].w));
}
__device__ __forceinline__ void pin(FootRaw<true, false>& R)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) asm volatile("" : "+v"(R.h[i].x), "+v"(R.h[i].y));
}
template <bool CELL>
__device__ __forceinline__ void pin(FootRaw<false, CELL>& R)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) asm volatile("" : "+v"(R.c[i].x), "+v"(R.c[i].y), "+v"(R.c[i].z), "+v"(R.c[i].w));
}
__device__ __forceinline__ void pin(Foot& F)
{
    // one 4-register operand per corner: the corner stays the register
    // quadruple its load wrote (no copies that would wait for the load)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f32x4 v = {F.c[i].x, F.c[i].y, F.c[i].z, F.c[i].w};
        asm volatile("" : "+v"(v));
        F.c[i] = make_float4(v.x, v.y, v.z, v.w);
    }
}

template <bool FP16, bool CELL>
__device__ __forceinline__ Foot load_foot(const void* __restrict__ lut, int N, const Loc& L)
{
    return decode<FP16, CELL>(load_raw<FP16, CELL>(lut, N, L));
}

// The arithmetic from a loaded footprint to a result fuses a multiply into an
// add only where one source expression holds both (fp contract(on) in each
// function below), never across statements as the code generator would
// choose it: every kernel that calls these functions then gives the same
// bits for the same inputs, whatever code surrounds the call.

// Cubic Hermite basis on [0,1], Eq. (3): only H1, H0d, H1d are needed
// (H0 = 1 - H1) plus first derivatives (H0' = -H1').
struct Basis1 {
    float h1, h0d, h1d;      // H1, H0^d, H1^d
    float d1, d0d, d1d;      // H1', (H0^d)', (H1^d)'
};

__device__ __forceinline__ Basis1 basis1(float s)
{
#pragma clang fp contract(on)
    Basis1 B;
    const float s2 = s * s;
    B.h1 = s2 * (3.0f - 2.0f * s);          // -2s^3 + 3s^2
    B.h0d = s * (s - 1.0f) * (s - 1.0f);    // s^3 - 2s^2 + s
    B.h1d = s2 * (s - 1.0f);                // s^3 - s^2
    B.d1 = 6.0f * s * (1.0f - s);           // -6s^2 + 6s
    B.d0d = (3.0f * s - 1.0f) * (s - 1.0f); // 3s^2 - 4s + 1
    B.d1d = s * (3.0f * s - 2.0f);          // 3s^2 - 2s
    return B;
}

struct Patch {
    float r, rs, rt;  // value and derivatives in the local (s, t); r_u = N rs
};

// Eq. (4) and its s, t derivatives, evaluated in difference form: every
// corner difference (exact in FP32 for nearby values) is taken before it is
// weighted, so chart derivatives keep full relative accuracy at large N.
__device__ __forceinline__ Patch hermite(const Foot& F, float s, float t)
{
#pragma clang fp contract(on)
    const Basis1 S = basis1(s), T = basis1(t);
    const float4 c00 = F.c[0], c10 = F.c[1], c01 = F.c[2], c11 = F.c[3];
    // differences along s (rows j = 0, 1) and along t (columns i = 0, 1)
    const float dsR0 = c10.x - c00.x, dsR1 = c11.x - c01.x;
    const float dtR0 = c01.x - c00.x;
    const float dtU0 = c01.y - c00.y, dtU1 = c11.y - c10.y;
    const float dsV0 = c10.z - c00.z, dsV1 = c11.z - c01.z;
    // f_j(s): Hermite in s of (r, r_u h) on row j; g_j(s): of (r_v h, r_uv h^2)
    const float f0 = c00.x + S.h1 * dsR0 + S.h0d * c00.y + S.h1d * c10.y;
    const float df = dtR0 + S.h1 * (dsR1 - dsR0) + S.h0d * dtU0 + S.h1d * dtU1;  // f1 - f0
    const float g0 = c00.z + S.h1 * dsV0 + S.h0d * c00.w + S.h1d * c10.w;
    const float g1 = c01.z + S.h1 * dsV1 + S.h0d * c01.w + S.h1d * c11.w;
    const float f0s = S.d1 * dsR0 + S.d0d * c00.y + S.d1d * c10.y;
    const float f1s = S.d1 * dsR1 + S.d0d * c01.y + S.d1d * c11.y;
    const float g0s = S.d1 * dsV0 + S.d0d * c00.w + S.d1d * c10.w;
    const float g1s = S.d1 * dsV1 + S.d0d * c01.w + S.d1d * c11.w;
    Patch P;
    P.r = f0 + T.h1 * df + T.h0d * g0 + T.h1d * g1;
    P.rs = f0s + T.h1 * (f1s - f0s) + T.h0d * g0s + T.h1d * g1s;
    P.rt = T.d1 * df + T.d0d * g0 + T.d1d * g1;
    return P;
}

struct Patch2 {
    float r, rs, rt, rss, rst, rtt;  // value, first and second local derivatives
};

// Eq. (4) with first and second derivatives in (s, t) (difference form as in
// hermite()); the second derivatives feed the direction gradient of the
// backward.  H1'' = 6 - 12s, (H0^d)'' = 6s - 4, (H1^d)'' = 6s - 2.
__device__ __forceinline__ Patch2 hermite2(const Foot& F, float s, float t)
{
#pragma clang fp contract(on)
    const Basis1 S = basis1(s), T = basis1(t);
    const float e1s = 6.0f - 12.0f * s, e0ds = 6.0f * s - 4.0f, e1ds = 6.0f * s - 2.0f;
    const float e1t = 6.0f - 12.0f * t, e0dt = 6.0f * t - 4.0f, e1dt = 6.0f * t - 2.0f;
    const float4 c00 = F.c[0], c10 = F.c[1], c01 = F.c[2], c11 = F.c[3];
    const float dsR0 = c10.x - c00.x, dsR1 = c11.x - c01.x;
    const float dtR0 = c01.x - c00.x;
    const float dtU0 = c01.y - c00.y, dtU1 = c11.y - c10.y;
    const float dsV0 = c10.z - c00.z, dsV1 = c11.z - c01.z;
    const float f0 = c00.x + S.h1 * dsR0 + S.h0d * c00.y + S.h1d * c10.y;
    const float df = dtR0 + S.h1 * (dsR1 - dsR0) + S.h0d * dtU0 + S.h1d * dtU1;
    const float g0 = c00.z + S.h1 * dsV0 + S.h0d * c00.w + S.h1d * c10.w;
    const float g1 = c01.z + S.h1 * dsV1 + S.h0d * c01.w + S.h1d * c11.w;
    const float f0s = S.d1 * dsR0 + S.d0d * c00.y + S.d1d * c10.y;
    const float f1s = S.d1 * dsR1 + S.d0d * c01.y + S.d1d * c11.y;
    const float g0s = S.d1 * dsV0 + S.d0d * c00.w + S.d1d * c10.w;
    const float g1s = S.d1 * dsV1 + S.d0d * c01.w + S.d1d * c11.w;
    const float f0ss = e1s * dsR0 + e0ds * c00.y + e1ds * c10.y;
    const float f1ss = e1s * dsR1 + e0ds * c01.y + e1ds * c11.y;
    const float g0ss = e1s * dsV0 + e0ds * c00.w + e1ds * c10.w;
    const float g1ss = e1s * dsV1 + e0ds * c01.w + e1ds * c11.w;
    Patch2 P;
    P.r = f0 + T.h1 * df + T.h0d * g0 + T.h1d * g1;
    P.rs = f0s + T.h1 * (f1s - f0s) + T.h0d * g0s + T.h1d * g1s;
    P.rt = T.d1 * df + T.d0d * g0 + T.d1d * g1;
    P.rss = f0ss + T.h1 * (f1ss - f0ss) + T.h0d * g0ss + T.h1d * g1ss;
    P.rst = T.d1 * (f1s - f0s) + T.d0d * g0s + T.d1d * g1s;
    P.rtt = e1t * df + e0dt * g0 + e1dt * g1;
    return P;
}

// Per-face frame as signed axis vectors: M, S, T of the hardware cube map.
__device__ __forceinline__ void frame_of(int face, float3& M, float3& S, float3& T)
{
    switch (face) {
    case 0: M = make_float3(1, 0, 0); S = make_float3(0, 0, -1); T = make_float3(0, -1, 0); break;
    case 1: M = make_float3(-1, 0, 0); S = make_float3(0, 0, 1); T = make_float3(0, -1, 0); break;
    case 2: M = make_float3(0, 1, 0); S = make_float3(1, 0, 0); T = make_float3(0, 0, 1); break;
    case 3: M = make_float3(0, -1, 0); S = make_float3(1, 0, 0); T = make_float3(0, 0, -1); break;
    case 4: M = make_float3(0, 0, 1); S = make_float3(1, 0, 0); T = make_float3(0, -1, 0); break;
    default: M = make_float3(0, 0, -1); S = make_float3(-1, 0, 0); T = make_float3(0, -1, 0); break;
    }
}

// Ambient spherical gradient from chart derivatives (r_u, r_v), closed form
// of the Sec. 3.4 metric solve.  Per face: M, S, T are signed axis vectors.
template <bool FAST>
__device__ __forceinline__ float3 transport_t(int face, float a, float b, float ru, float rv)
{
#pragma clang fp contract(on)
    const float rho2 = 1.0f + a * a + b * b;
    const float rho = FAST ? __builtin_amdgcn_sqrtf(rho2) : sqrtf(rho2);
    const float k = 0.5f * rho;
    const float gu = k * ru, gv = k * rv;
    const float gm = -(a * gu + b * gv);  // component along M
    // g = gu S + gv T + gm M
    switch (face) {
    case 0: return make_float3(gm, -gv, -gu);   // M=+x S=-z T=-y
    case 1: return make_float3(-gm, -gv, gu);   // M=-x S=+z T=-y
    case 2: return make_float3(gu, gm, gv);     // M=+y S=+x T=+z
    case 3: return make_float3(gu, -gm, -gv);   // M=-y S=+x T=-z
    case 4: return make_float3(gu, -gv, gm);    // M=+z S=+x T=-y
    default: return make_float3(-gu, -gv, -gm); // M=-z S=-x T=-y
    }
}

__device__ __forceinline__ float3 transport(int face, float a, float b, float ru, float rv)
{
    return transport_t<false>(face, a, b, ru, rv);
}

// Eq. (10)
__device__ __forceinline__ float3 normal_of(float R, float x, float y, float z, float3 g)
{
#pragma clang fp contract(on)
    const float3 w = unit_dir(x, y, z);
    const float mx = R * w.x - g.x, my = R * w.y - g.y, mz = R * w.z - g.z;
    const float in = rsqrtf(mx * mx + my * my + mz * mz);
    return make_float3(mx * in, my * in, mz * in);
}

// The query's arithmetic after its loads: (r, grad r) from the footprint of
// a valid location.
template <bool FAST = false>
__device__ __forceinline__ float4 query_eval(const Foot& F, const Loc& L, int N)
{
#pragma clang fp contract(on)
    const Patch P = hermite(F, L.s, L.t);
    const float Nf = (float)N;
    const float3 g = transport_t<FAST>(L.face, L.a, L.b, Nf * P.rs, Nf * P.rt);
    return make_float4(P.r, g.x, g.y, g.z);
}

// Full query: returns (R, gx, gy, gz); NaN for an invalid direction.
template <bool FP16, bool CELL, bool FAST = false>
__device__ __forceinline__ float4 query_one(const void* __restrict__ lut, int N, float x, float y, float z)
{
    const Loc L = locate_t<FAST>(x, y, z, N);
    if (L.face < 0) return make_float4(__builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""), __builtin_nanf(""));
    const Foot F = load_foot<FP16, CELL>(lut, N, L);
    return query_eval<FAST>(F, L, N);
}

// The same query in two halves with no branch between them, for kernels that
// issue the loads of several queries before any of their arithmetic:
// query_load reads the footprint of L's cell (of face 0 for an invalid
// direction: i0, j0 are always clamped to [0, N], so the address stays in the
// LUT), query_finish on its decoded form gives query_one's result bit for bit.
template <bool FP16, bool CELL>
__device__ __forceinline__ FootRaw<FP16, CELL> query_load(const void* __restrict__ lut, int N, const Loc& L)
{
    Loc Ls = L;
    Ls.face = L.face < 0 ? 0 : L.face;
    return load_raw<FP16, CELL>(lut, N, Ls);
}

__device__ __forceinline__ float4 query_finish(const Foot& F, const Loc& L, int N)
{
    const float4 r = query_eval(F, L, N);
    const float nan = __builtin_nanf("");
    return L.face < 0 ? make_float4(nan, nan, nan, nan) : r;
}

// Rendered radius (Sec. 3.1) from (r, grad r): R = s r, or for a signed
// function R = s |r| with gradient s sign(r) grad r (Sec. 3.4, after Eq. 10;
// sign(0) = 0).  *sgn gets sign(r); NaN input stays NaN.
__device__ __forceinline__ float4 rendered(float4 q, float scale, bool is_signed, int* sgn)
{
#pragma clang fp contract(on)
    const float r = q.x;
    const int sg = r > 0.0f ? 1 : (r < 0.0f ? -1 : 0);
    *sgn = sg;
    const float k = is_signed ? scale * (float)sg : scale;
    const float R = is_signed ? scale * fabsf(r) : scale * r;
    if (r != r) return q;
    return make_float4(R, k * q.y, k * q.z, k * q.w);
}

}  // namespace shm
