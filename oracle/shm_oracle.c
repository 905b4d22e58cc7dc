/*
 * shm_oracle.c -- plain FP64 CPU oracle for Spherical Hermite Maps
 * (Abouagour & Garyfallidis, arXiv 2602.20063).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: the
 * HIP library never includes, links, loads or calls it, and it includes
 * nothing from the HIP library.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark use it.
 *
 * Everything here is written for a reader who checks it against the paper by
 * eye: no blocking, no fusion, no reordering beyond what the equations state.
 * All arithmetic is IEEE double, the integer decisions of a query (face and
 * cell) included: they are taken on the exact FP64 coordinate of the FP32
 * input.  An implementation that decides in single precision may pick the
 * neighbouring cell where that coordinate lies within a few FP32 ulps of a
 * cell edge; such ties are counted by the tests, not hidden here.  (The one
 * FP32 decision left is the adaptive bisection budget of the ray caster, a
 * count the paper leaves open, documented at bisect_budget().)
 *
 * Derivatives needed by the bake (chart derivatives r_u, r_v, r_uv) and by the
 * direction gradient of the backward are obtained with hyper-dual numbers
 * (Fike & Alonso, AIAA 2011-886): exact first and mixed second derivatives,
 * no step size.  A hyper-dual x = v + a e1 + b e2 + ab e1e2, e1^2 = e2^2 = 0.
 *
 * Section / equation references are to the paper:
 *   Sec. 3.1 (Eq. 1)       star-shaped surface, implicit F, ray bracket, root refinement
 *   Sec. 3.2               padded cubemap parameterisation, gutter texels
 *   Sec. 3.3 Eq. (2)       texel storage (r, r_u h, r_v h, r_uv h^2)
 *   Sec. 3.3 Alg. 1        bake per face
 *   Sec. 3.3 Eqs. (3)-(5)  Hermite basis, reconstruction, chart derivatives
 *   Sec. 3.4 Eqs. (6)-(10) tangents, metric tensor, Cramer solve, normal
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   face table        standard hardware cubemap convention (+X,-X,+Y,-Y,+Z,-Z)
 *   face tie-break    |x| >= |y|, |z| -> X; else |y| >= |z| -> Y; else Z;
 *                     component >= 0 -> positive face; applied to the raw input
 *   texel centres     cell-centred: padded index p in 0..N+1 sits at u=(p-1/2)/N
 *   gutter            texel-centre direction on the extended face plane
 *   real SH           orthonormal, no Condon-Shortley phase, k = l^2 + l + m
 *   det G clamp       max(det G, 1e-12)
 *   trace schedule    march K, bisect B, safeguarded Newton M, fixed counts
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* hyper-dual numbers                                                        */
/* ------------------------------------------------------------------------ */
typedef struct { double v, a, b, ab; } hd;

static hd hc(double x) { hd r = {x, 0.0, 0.0, 0.0}; return r; }
static hd hadd(hd x, hd y) { hd r = {x.v + y.v, x.a + y.a, x.b + y.b, x.ab + y.ab}; return r; }
static hd hsub(hd x, hd y) { hd r = {x.v - y.v, x.a - y.a, x.b - y.b, x.ab - y.ab}; return r; }
static hd hscale(hd x, double c) { hd r = {x.v * c, x.a * c, x.b * c, x.ab * c}; return r; }
static hd hmul(hd x, hd y)
{
    hd r;
    r.v = x.v * y.v;
    r.a = x.a * y.v + x.v * y.a;
    r.b = x.b * y.v + x.v * y.b;
    r.ab = x.ab * y.v + x.a * y.b + x.b * y.a + x.v * y.ab;
    return r;
}
/* g(x) for a scalar function with value f, first derivative f1, second f2 */
static hd hfun(hd x, double f, double f1, double f2)
{
    hd r;
    r.v = f;
    r.a = f1 * x.a;
    r.b = f1 * x.b;
    r.ab = f1 * x.ab + f2 * x.a * x.b;
    return r;
}
static hd hsqrt(hd x) { double s = sqrt(x.v); return hfun(x, s, 0.5 / s, -0.25 / (s * x.v)); }
static hd hinv(hd x) { double i = 1.0 / x.v; return hfun(x, i, -i * i, 2.0 * i * i * i); }
static hd hdiv(hd x, hd y) { return hmul(x, hinv(y)); }
static hd hexp(hd x) { double e = exp(x.v); return hfun(x, e, e, e); }

/* ------------------------------------------------------------------------ */
/* cubemap face table (Sec. 3.2: faces "align with GPU cubemap hardware")    */
/* d / |major| = M + sc*S + tc*T, u = (sc+1)/2, v = (tc+1)/2                 */
/* ------------------------------------------------------------------------ */
static const double FM[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
static const double FS[6][3] = {{0, 0, -1}, {0, 0, 1}, {1, 0, 0}, {1, 0, 0}, {1, 0, 0}, {-1, 0, 0}};
static const double FT[6][3] = {{0, -1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}, {0, -1, 0}, {0, -1, 0}};

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Face selection on the raw components (exact in any precision). */
static int face_select(double x, double y, double z)
{
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) return -1;
    if (x == 0.0 && y == 0.0 && z == 0.0) return -1;
    double ax = fabs(x), ay = fabs(y), az = fabs(z);
    if (ax >= ay && ax >= az) return x >= 0.0 ? 0 : 1;
    if (ay >= az) return y >= 0.0 ? 2 : 3;
    return z >= 0.0 ? 4 : 5;
}

/* Location of a query inside the padded face: the face, the cell (i0, j0)
 * whose corners are padded texels (i0+{0,1}, j0+{0,1}), and the local
 * coordinates (s, t) of Eq. (4).  Padded texel p has its centre at
 * u = (p - 1/2)/N, so the continuous padded coordinate is f = u N + 1/2 and
 * i0 = min(floor(f), N), s = f - i0 (u = 1 exactly belongs to the last
 * cell).  Everything is FP64: for an FP32 input the coordinate f carries a
 * relative error of a few FP64 ulps, so the cell is the exact one unless f
 * is within ~1e-15 of an integer. */
typedef struct {
    int face, i0, j0;
    double a, b;   /* sc/ma, tc/ma in [-1, 1] */
    double s, t;
} loc_t;

static int locate(const double d[3], int N, loc_t* L)
{
    int f = face_select(d[0], d[1], d[2]);
    L->face = f;
    if (f < 0) return 0;
    double sc = dot3(d, FS[f]), tc = dot3(d, FT[f]), ma = dot3(d, FM[f]);
    L->a = sc / ma;
    L->b = tc / ma;
    double fu = (L->a + 1.0) * 0.5 * (double)N + 0.5;
    double fv = (L->b + 1.0) * 0.5 * (double)N + 0.5;
    int i0 = (int)floor(fu), j0 = (int)floor(fv);
    if (i0 > N) i0 = N;
    if (j0 > N) j0 = N;
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    L->i0 = i0;
    L->j0 = j0;
    L->s = fu - (double)i0;
    L->t = fv - (double)j0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Hermite basis, Eq. (3), and derivatives                                   */
/* ------------------------------------------------------------------------ */
/* Hb[0..3] = H0, H1, H0d, H1d;  Hd[0..3] = their first derivatives */
static void hermite_hd(hd s, hd Hb[4], hd Hd[4])
{
    hd s2 = hmul(s, s), s3 = hmul(s2, s);
    Hb[0] = hadd(hsub(hscale(s3, 2.0), hscale(s2, 3.0)), hc(1.0));   /* 2s^3 - 3s^2 + 1 */
    Hb[1] = hadd(hscale(s3, -2.0), hscale(s2, 3.0));                 /* -2s^3 + 3s^2    */
    Hb[2] = hadd(hsub(s3, hscale(s2, 2.0)), s);                      /* s^3 - 2s^2 + s  */
    Hb[3] = hsub(s3, s2);                                            /* s^3 - s^2       */
    Hd[0] = hsub(hscale(s2, 6.0), hscale(s, 6.0));                   /* 6s^2 - 6s       */
    Hd[1] = hadd(hscale(s2, -6.0), hscale(s, 6.0));                  /* -6s^2 + 6s      */
    Hd[2] = hadd(hsub(hscale(s2, 3.0), hscale(s, 4.0)), hc(1.0));    /* 3s^2 - 4s + 1   */
    Hd[3] = hsub(hscale(s2, 3.0), hscale(s, 2.0));                   /* 3s^2 - 2s       */
}

ORC_API void orc_hermite_basis(double s, double* out8)
{
    hd Hb[4], Hd[4];
    hermite_hd(hc(s), Hb, Hd);
    for (int k = 0; k < 4; ++k) { out8[k] = Hb[k].v; out8[4 + k] = Hd[k].v; }
}

/* LUT indexing: lut[((face*(N+2) + q)*(N+2) + p)*4 + ch], q = v row, p = u column */
static size_t texel_index(int N, int face, int p, int q)
{
    return (((size_t)face * (size_t)(N + 2) + (size_t)q) * (size_t)(N + 2) + (size_t)p) * 4u;
}

/* Eq. (4) and Eq. (5): value and chart derivatives from the 16 scalars of the
 * 2x2 footprint.  C[j][i][ch] is corner (i0+i, j0+j), channels
 * (r, r_u h, r_v h, r_uv h^2).  Derivatives w.r.t. u carry the factor 1/h = N. */
static void reconstruct_hd(const double C[2][2][4], int N, hd s, hd t, hd* r, hd* ru, hd* rv)
{
    hd Hs[4], Hds[4], Ht[4], Hdt[4];
    hermite_hd(s, Hs, Hds);
    hermite_hd(t, Ht, Hdt);
    hd acc = hc(0.0), accu = hc(0.0), accv = hc(0.0);
    for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i) {
            const double* c = C[j][i];
            /* H_i, H^d_i in s; H_j, H^d_j in t */
            hd Hi = Hs[i], Hdi = Hs[2 + i], Hj = Ht[j], Hdj = Ht[2 + j];
            hd dHi = Hds[i], dHdi = Hds[2 + i], dHj = Hdt[j], dHdj = Hdt[2 + j];
            acc = hadd(acc, hscale(hmul(Hi, Hj), c[0]));
            acc = hadd(acc, hscale(hmul(Hdi, Hj), c[1]));
            acc = hadd(acc, hscale(hmul(Hi, Hdj), c[2]));
            acc = hadd(acc, hscale(hmul(Hdi, Hdj), c[3]));
            accu = hadd(accu, hscale(hmul(dHi, Hj), c[0]));
            accu = hadd(accu, hscale(hmul(dHdi, Hj), c[1]));
            accu = hadd(accu, hscale(hmul(dHi, Hdj), c[2]));
            accu = hadd(accu, hscale(hmul(dHdi, Hdj), c[3]));
            accv = hadd(accv, hscale(hmul(Hi, dHj), c[0]));
            accv = hadd(accv, hscale(hmul(Hdi, dHj), c[1]));
            accv = hadd(accv, hscale(hmul(Hi, dHdj), c[2]));
            accv = hadd(accv, hscale(hmul(Hdi, dHdj), c[3]));
        }
    *r = acc;
    *ru = hscale(accu, (double)N);
    *rv = hscale(accv, (double)N);
}

static void gather_corners(const double* lut, int N, int face, int i0, int j0, double C[2][2][4])
{
    for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i) {
            const double* src = lut + texel_index(N, face, i0 + i, j0 + j);
            for (int ch = 0; ch < 4; ++ch) C[j][i][ch] = src[ch];
        }
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.4: chart derivatives -> spherical gradient -> normal               */
/* ------------------------------------------------------------------------ */
typedef struct {
    hd R, ru, rv;
    hd grad[3];
    hd w[3];      /* unit direction omega */
    hd detG;
    int clamped;
} transport_t;

/* Eq. (6)-(9): e_xi = (I - w w^T) / |w~| * d w~/d xi with d w~/du = 2S,
 * d w~/dv = 2T (w~ = M + (2u-1) S + (2v-1) T); G = [e_i . e_j]; Cramer. */
static void transport_hd(int face, hd a, hd b, hd ru, hd rv, transport_t* T)
{
    hd wt[3], w[3], e1[3], e2[3];
    for (int k = 0; k < 3; ++k)
        wt[k] = hadd(hadd(hc(FM[face][k]), hscale(a, FS[face][k])), hscale(b, FT[face][k]));
    hd rho = hsqrt(hadd(hadd(hmul(wt[0], wt[0]), hmul(wt[1], wt[1])), hmul(wt[2], wt[2])));
    hd irho = hinv(rho);
    for (int k = 0; k < 3; ++k) w[k] = hmul(wt[k], irho);
    /* w . dwt/du = 2 (w . S);  e1 = (2S - w (w . 2S)) / rho */
    hd wS = hc(0.0), wT = hc(0.0);
    for (int k = 0; k < 3; ++k) {
        wS = hadd(wS, hscale(w[k], 2.0 * FS[face][k]));
        wT = hadd(wT, hscale(w[k], 2.0 * FT[face][k]));
    }
    for (int k = 0; k < 3; ++k) {
        e1[k] = hmul(hsub(hc(2.0 * FS[face][k]), hmul(w[k], wS)), irho);
        e2[k] = hmul(hsub(hc(2.0 * FT[face][k]), hmul(w[k], wT)), irho);
    }
    hd g11 = hc(0.0), g12 = hc(0.0), g22 = hc(0.0);
    for (int k = 0; k < 3; ++k) {
        g11 = hadd(g11, hmul(e1[k], e1[k]));
        g12 = hadd(g12, hmul(e1[k], e2[k]));
        g22 = hadd(g22, hmul(e2[k], e2[k]));
    }
    hd det = hsub(hmul(g11, g22), hmul(g12, g12));
    T->detG = det;
    T->clamped = 0;
    if (!(det.v >= 1e-12)) { det = hc(1e-12); T->clamped = 1; }
    hd idet = hinv(det);
    hd alpha = hmul(hsub(hmul(g22, ru), hmul(g12, rv)), idet);
    hd beta = hmul(hsub(hmul(g11, rv), hmul(g12, ru)), idet);
    for (int k = 0; k < 3; ++k) {
        T->grad[k] = hadd(hmul(alpha, e1[k]), hmul(beta, e2[k]));
        T->w[k] = w[k];
    }
    T->ru = ru;
    T->rv = rv;
}

/* Closed form of the same gradient (used only as a cross-check):
 * grad = (rho/2) [ r_u (S - a M) + r_v (T - b M) ],  rho = sqrt(1 + a^2 + b^2). */
static void transport_closed(int face, double a, double b, double ru, double rv, double g[3])
{
    double rho = sqrt(1.0 + a * a + b * b);
    for (int k = 0; k < 3; ++k)
        g[k] = 0.5 * rho * (ru * (FS[face][k] - a * FM[face][k]) + rv * (FT[face][k] - b * FM[face][k]));
}

/* Eq. (10) */
static void normal_of(double R, const double w[3], const double g[3], double n[3])
{
    double m[3], len = 0.0;
    for (int k = 0; k < 3; ++k) { m[k] = R * w[k] - g[k]; len += m[k] * m[k]; }
    len = sqrt(len);
    for (int k = 0; k < 3; ++k) n[k] = m[k] / len;
}

/* One full query with direction d = d0 + e1 * dd (hyper-dual tangent on e1);
 * face and cell are decided from d0 only.  Returns 0 for an invalid d0. */
typedef struct {
    loc_t L;
    transport_t T;
    hd R;
} query_t;

static int query_hd(const double* lut, int N, const double d0[3], const double dd[3], query_t* Q)
{
    if (!locate(d0, N, &Q->L)) return 0;
    int f = Q->L.face;
    hd d[3];
    for (int k = 0; k < 3; ++k) { d[k] = hc(d0[k]); d[k].a = dd ? dd[k] : 0.0; }
    /* a = (d.S)/(d.M), b = (d.T)/(d.M): sc, tc of the cubemap table */
    hd dS = hc(0.0), dT = hc(0.0), dM = hc(0.0);
    for (int k = 0; k < 3; ++k) {
        dS = hadd(dS, hscale(d[k], FS[f][k]));
        dT = hadd(dT, hscale(d[k], FT[f][k]));
        dM = hadd(dM, hscale(d[k], FM[f][k]));
    }
    hd a = hdiv(dS, dM), b = hdiv(dT, dM);
    /* s = (a+1)/2 N + 1/2 - i0 (face and cell frozen) */
    hd s = hsub(hadd(hscale(hadd(a, hc(1.0)), 0.5 * N), hc(0.5)), hc((double)Q->L.i0));
    hd t = hsub(hadd(hscale(hadd(b, hc(1.0)), 0.5 * N), hc(0.5)), hc((double)Q->L.j0));
    double C[2][2][4];
    gather_corners(lut, N, f, Q->L.i0, Q->L.j0, C);
    hd r, ru, rv;
    reconstruct_hd(C, N, s, t, &r, &ru, &rv);
    transport_hd(f, a, b, ru, rv, &Q->T);
    Q->R = r;
    return 1;
}

/* Same as query_hd but on a caller-chosen face (d . M_face > 0 required),
 * cell decided in FP64 and clamped to the padded grid; used to evaluate both
 * sides of a face seam. */
static int query_on_face(const double* lut, int N, int f, const double d0[3], query_t* Q)
{
    double sc = dot3(d0, FS[f]), tc = dot3(d0, FT[f]), ma = dot3(d0, FM[f]);
    if (!(ma > 0.0)) return 0;
    loc_t* L = &Q->L;
    L->face = f;
    L->a = sc / ma;
    L->b = tc / ma;
    double fu = (L->a + 1.0) * 0.5 * (double)N + 0.5, fv = (L->b + 1.0) * 0.5 * (double)N + 0.5;
    int i0 = (int)floor(fu), j0 = (int)floor(fv);
    if (i0 > N) i0 = N;
    if (j0 > N) j0 = N;
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    L->i0 = i0;
    L->j0 = j0;
    L->s = fu - i0;
    L->t = fv - j0;
    double C[2][2][4];
    gather_corners(lut, N, f, i0, j0, C);
    hd r, ru, rv;
    reconstruct_hd(C, N, hc(L->s), hc(L->t), &r, &ru, &rv);
    transport_hd(f, hc(L->a), hc(L->b), ru, rv, &Q->T);
    Q->R = r;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Public query API                                                          */
/* ------------------------------------------------------------------------ */

/* Face / cell / local coordinates of each query (all FP64). */
ORC_API void orc_locate(const float* dirs, int64_t Q, int N, int32_t* face, int32_t* i0, int32_t* j0, double* s, double* t)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        double d[3] = {dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2]};
        loc_t L;
        if (!locate(d, N, &L)) { face[q] = -1; i0[q] = j0[q] = -1; s[q] = t[q] = NAN; continue; }
        face[q] = L.face; i0[q] = L.i0; j0[q] = L.j0; s[q] = L.s; t[q] = L.t;
    }
}

/* Value + spherical gradient (+ normal) of each query, Sec. 3.3-3.4.
 * out[q] = (R, gx, gy, gz); normal may be NULL.
 * closed_form = 0: the paper's route (e1, e2, G, Cramer); 1: closed form.
 * Invalid directions (zero / non-finite) give NaN. */
ORC_API void orc_query(const double* lut, int N, const float* dirs, int64_t Q, int closed_form, double* out, double* normal)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        double d[3] = {dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2]};
        query_t QR;
        if (!query_hd(lut, N, d, NULL, &QR)) {
            for (int k = 0; k < 4; ++k) out[4 * q + k] = NAN;
            if (normal) for (int k = 0; k < 3; ++k) normal[3 * q + k] = NAN;
            continue;
        }
        double g[3], w[3];
        if (closed_form) transport_closed(QR.L.face, QR.L.a, QR.L.b, QR.T.ru.v, QR.T.rv.v, g);
        else for (int k = 0; k < 3; ++k) g[k] = QR.T.grad[k].v;
        for (int k = 0; k < 3; ++k) w[k] = QR.T.w[k].v;
        out[4 * q] = QR.R.v;
        for (int k = 0; k < 3; ++k) out[4 * q + 1 + k] = g[k];
        if (normal) normal_of(QR.R.v, w, g, normal + 3 * q);
    }
}

/* Rendered radius of Sec. 3.1 for a user scale s > 0: R = s r for a
 * nonnegative function; for a signed one R = s |r|, whose gradient is
 * s sign(r) grad r by the chain rule of the absolute value (Sec. 3.4, after
 * Eq. 10), with sign(0) = 0.  The normal is Eq. 10 with these R, grad R. */
static double rendered(double r, const double gr[3], double s, int signed_, double g[3], int* sgn)
{
    int sg = r > 0.0 ? 1 : (r < 0.0 ? -1 : 0);
    double k = signed_ ? s * sg : s;
    for (int i = 0; i < 3; ++i) g[i] = k * gr[i];
    if (sgn) *sgn = sg;
    return signed_ ? s * fabs(r) : s * r;
}

/* Query of the rendered radius: out (R, grad R), normal (Eq. 10), and the
 * sign of r (+1, -1, 0; 0 also for an invalid direction). */
ORC_API void orc_query_scaled(const double* lut, int N, const float* dirs, int64_t Q, double scale, int signed_,
                              double* out, double* normal, int8_t* sign)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        double d[3] = {dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2]};
        query_t QR;
        if (!query_hd(lut, N, d, NULL, &QR)) {
            for (int k = 0; k < 4; ++k) out[4 * q + k] = NAN;
            if (normal) for (int k = 0; k < 3; ++k) normal[3 * q + k] = NAN;
            if (sign) sign[q] = 0;
            continue;
        }
        double gr[3], g[3], w[3];
        int sg;
        for (int k = 0; k < 3; ++k) { gr[k] = QR.T.grad[k].v; w[k] = QR.T.w[k].v; }
        double R = rendered(QR.R.v, gr, scale, signed_, g, &sg);
        out[4 * q] = R;
        for (int k = 0; k < 3; ++k) out[4 * q + 1 + k] = g[k];
        if (normal) normal_of(R, w, g, normal + 3 * q);
        if (sign) sign[q] = (int8_t)sg;
    }
}

/* FP64 directions (finite-difference pins, truth-level comparisons).  face_forced < 0: own face; else evaluate on that face. */
ORC_API void orc_query_f64(const double* lut, int N, const double* dirs, int64_t Q, int face_forced, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        const double* d = dirs + 3 * q;
        query_t QR;
        int ok = face_forced < 0 ? query_hd(lut, N, d, NULL, &QR) : query_on_face(lut, N, face_forced, d, &QR);
        if (!ok) { for (int k = 0; k < 4; ++k) out[4 * q + k] = NAN; continue; }
        out[4 * q] = QR.R.v;
        for (int k = 0; k < 3; ++k) out[4 * q + 1 + k] = QR.T.grad[k].v;
    }
}

/* Diagnostics per query: (r, r_u, r_v, det G, clamped, a, b, w_x, w_y, w_z) */
ORC_API void orc_query_chart(const double* lut, int N, const float* dirs, int64_t Q, double* out10)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        double d[3] = {dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2]};
        query_t QR;
        double* o = out10 + 10 * q;
        if (!query_hd(lut, N, d, NULL, &QR)) { for (int k = 0; k < 10; ++k) o[k] = NAN; continue; }
        o[0] = QR.R.v; o[1] = QR.T.ru.v; o[2] = QR.T.rv.v; o[3] = QR.T.detG.v; o[4] = QR.T.clamped;
        o[5] = QR.L.a; o[6] = QR.L.b; o[7] = QR.T.w[0].v; o[8] = QR.T.w[1].v; o[9] = QR.T.w[2].v;
    }
}

/* Reconstruction at an explicit (face, cell, s, t): out5 = (r, r_u, r_v) plus
 * the spherical gradient is not formed here (cell-level pin tests). */
ORC_API void orc_reconstruct(const double* lut, int N, int face, int i0, int j0, double s, double t, double* out3)
{
    double C[2][2][4];
    gather_corners(lut, N, face, i0, j0, C);
    hd r, ru, rv;
    reconstruct_hd(C, N, hc(s), hc(t), &r, &ru, &rv);
    out3[0] = r.v; out3[1] = ru.v; out3[2] = rv.v;
}

/* Batched queries: object o owns lut[lut_off[o]*4 ...] with face size Ns[o]
 * and queries [q_begin[o], q_begin[o] + q_count[o]).  No cross-object
 * interaction: each object is an independent single-object query. */
ORC_API void orc_query_objects(const double* lut, const int64_t* lut_off, const int32_t* Ns, const int64_t* q_begin,
                               const int64_t* q_count, int64_t n_obj, const float* dirs, double* out, double* normal)
{
    /* objects in parallel; the per-object loop inside runs on its thread */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t o = 0; o < n_obj; ++o)
        orc_query(lut + 4 * lut_off[o], Ns[o], dirs + 3 * q_begin[o], q_count[o], 0, out + 4 * q_begin[o],
                  normal ? normal + 3 * q_begin[o] : NULL);
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics (Cartesian, pole-free)                           */
/* Y_l0 = K_l0 Q_l^0(z);  Y_{l,+m} = sqrt2 K_lm Q_l^m(z) Re (x+iy)^m;        */
/* Y_{l,-m} = sqrt2 K_lm Q_l^m(z) Im (x+iy)^m,  Q_l^m = d^m P_l / dz^m,      */
/* K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).  Index k = l^2 + l + m.         */
/* ------------------------------------------------------------------------ */
#define ORC_LMAX 32

static void sh_hd(int L, hd x, hd y, hd z, hd* Y)
{
    hd A[ORC_LMAX + 1], B[ORC_LMAX + 1];
    A[0] = hc(1.0);
    B[0] = hc(0.0);
    for (int m = 1; m <= L; ++m) {
        A[m] = hsub(hmul(A[m - 1], x), hmul(B[m - 1], y));
        B[m] = hadd(hmul(A[m - 1], y), hmul(B[m - 1], x));
    }
    for (int m = 0; m <= L; ++m) {
        double qmm = 1.0; /* (2m-1)!! */
        for (int k = 1; k <= m; ++k) qmm *= (double)(2 * k - 1);
        hd Qm2 = hc(0.0), Qm1 = hc(0.0), Q = hc(0.0);
        for (int l = m; l <= L; ++l) {
            if (l == m) Q = hc(qmm);
            else if (l == m + 1) Q = hscale(z, (double)(2 * m + 1) * qmm);
            else Q = hscale(hsub(hscale(hmul(z, Qm1), (double)(2 * l - 1)), hscale(Qm2, (double)(l + m - 1))), 1.0 / (double)(l - m));
            double ratio = 1.0; /* (l-m)!/(l+m)! */
            for (int k = l - m + 1; k <= l + m; ++k) ratio /= (double)k;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * ratio);
            if (m == 0) Y[l * l + l] = hscale(Q, K);
            else {
                Y[l * l + l + m] = hscale(hmul(Q, A[m]), sqrt(2.0) * K);
                Y[l * l + l - m] = hscale(hmul(Q, B[m]), sqrt(2.0) * K);
            }
            Qm2 = Qm1;
            Qm1 = Q;
        }
    }
}

/* Basis values Y_k at unit directions: Y[q*(L+1)^2 + k] */
ORC_API void orc_sh_basis(int L, const double* dirs, int64_t Q, double* Y)
{
    int K = (L + 1) * (L + 1);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        hd Yh[(ORC_LMAX + 1) * (ORC_LMAX + 1)];
        sh_hd(L, hc(dirs[3 * q]), hc(dirs[3 * q + 1]), hc(dirs[3 * q + 2]), Yh);
        for (int k = 0; k < K; ++k) Y[q * K + k] = Yh[k].v;
    }
}

static hd sh_sum_hd(const double* c, int L, hd x, hd y, hd z)
{
    hd Y[(ORC_LMAX + 1) * (ORC_LMAX + 1)];
    sh_hd(L, x, y, z, Y);
    hd acc = hc(0.0);
    for (int k = 0; k < (L + 1) * (L + 1); ++k) acc = hadd(acc, hscale(Y[k], c[k]));
    return acc;
}

/* Truth: R = sum c_k Y_k(w) at w = d/|d| and the spherical gradient (the
 * ambient gradient of the 0-homogeneous extension R(x/|x|)), by hyper-dual
 * perturbation along the Cartesian axes.  out[q] = (R, gx, gy, gz). */
ORC_API void orc_sh_truth(const double* c, int L, const double* dirs, int64_t Q, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        double g[3];
        double Rv = 0.0;
        for (int pass = 0; pass < 3; ++pass) {
            hd x[3];
            for (int k = 0; k < 3; ++k) { x[k] = hc(dirs[3 * q + k]); x[k].a = (k == pass) ? 1.0 : 0.0; }
            hd n = hsqrt(hadd(hadd(hmul(x[0], x[0]), hmul(x[1], x[1])), hmul(x[2], x[2])));
            hd in = hinv(n);
            hd R = sh_sum_hd(c, L, hmul(x[0], in), hmul(x[1], in), hmul(x[2], in));
            g[pass] = R.a * n.v; /* gradient of the 0-homogeneous extension at the unit sphere */
            Rv = R.v;
        }
        out[4 * q] = Rv;
        for (int k = 0; k < 3; ++k) out[4 * q + 1 + k] = g[k];
    }
}

/* ------------------------------------------------------------------------ */
/* Bake, Alg. 1 (SH mode): every padded texel, gutter included, stores       */
/* (G, G_u h, G_v h, G_uv h^2) with G(u,v) = R(normalise(M+(2u-1)S+(2v-1)T)) */
/* ------------------------------------------------------------------------ */
typedef hd (*radial_fn)(const void* ctx, hd x, hd y, hd z);

static void bake_point(radial_fn fn, const void* ctx, int face, double u, double v, int N, double* out4)
{
    hd U = {u, 1.0, 0.0, 0.0}, V = {v, 0.0, 1.0, 0.0};
    hd A = hsub(hscale(U, 2.0), hc(1.0)), B = hsub(hscale(V, 2.0), hc(1.0));
    hd wt[3];
    for (int k = 0; k < 3; ++k) wt[k] = hadd(hadd(hc(FM[face][k]), hscale(A, FS[face][k])), hscale(B, FT[face][k]));
    hd rho = hsqrt(hadd(hadd(hmul(wt[0], wt[0]), hmul(wt[1], wt[1])), hmul(wt[2], wt[2])));
    hd ir = hinv(rho);
    hd G = fn(ctx, hmul(wt[0], ir), hmul(wt[1], ir), hmul(wt[2], ir));
    double h = 1.0 / (double)N;
    out4[0] = G.v;
    out4[1] = G.a * h;
    out4[2] = G.b * h;
    out4[3] = G.ab * h * h;
}

static void bake_face_all(radial_fn fn, const void* ctx, int N, double* lut)
{
    int P = N + 2;
#pragma omp parallel for collapse(2) schedule(static)
    for (int face = 0; face < 6; ++face)
        for (int q = 0; q < P; ++q)
            for (int p = 0; p < P; ++p) {
                double u = ((double)p - 0.5) / (double)N, v = ((double)q - 0.5) / (double)N;
                bake_point(fn, ctx, face, u, v, N, lut + texel_index(N, face, p, q));
            }
}

typedef struct { const double* c; int L; } sh_ctx;
static hd sh_fn(const void* ctx, hd x, hd y, hd z)
{
    const sh_ctx* S = (const sh_ctx*)ctx;
    return sh_sum_hd(S->c, S->L, x, y, z);
}

/* lut = [6][N+2][N+2][4] doubles */
ORC_API void orc_bake_sh(const double* c, int L, int N, double* lut)
{
    sh_ctx S = {c, L};
    bake_face_all(sh_fn, &S, N, lut);
}

/* Same channels at an arbitrary chart point (u, v) of a face. */
ORC_API void orc_bake_sh_point(const double* c, int L, int N, int face, double u, double v, double* out4)
{
    sh_ctx S = {c, L};
    bake_point(sh_fn, &S, face, u, v, N, out4);
}

/* Many glyphs: lut[o] = bake(c[o]) */
ORC_API void orc_bake_sh_many(const double* c, int L, int N, int64_t n_obj, double* lut)
{
    size_t K = (size_t)(L + 1) * (L + 1), T = (size_t)6 * (N + 2) * (N + 2) * 4;
    for (int64_t o = 0; o < n_obj; ++o) orc_bake_sh(c + o * K, L, N, lut + o * T);
}

/* Bumps on the sphere: R = base + sum_k amp_k exp((w . mu_k - 1) / width_k^2) */
typedef struct { const double* mu; const double* amp; const double* width; int K; double base; } bump_ctx;
static hd bump_fn(const void* ctx, hd x, hd y, hd z)
{
    const bump_ctx* B = (const bump_ctx*)ctx;
    hd acc = hc(B->base);
    for (int k = 0; k < B->K; ++k) {
        hd c = hadd(hadd(hscale(x, B->mu[3 * k]), hscale(y, B->mu[3 * k + 1])), hscale(z, B->mu[3 * k + 2]));
        hd e = hexp(hscale(hsub(c, hc(1.0)), 1.0 / (B->width[k] * B->width[k])));
        acc = hadd(acc, hscale(e, B->amp[k]));
    }
    return acc;
}

ORC_API void orc_bake_bumps(const double* mu, const double* amp, const double* width, int K, double base, int N, double* lut)
{
    bump_ctx B = {mu, amp, width, K, base};
    bake_face_all(bump_fn, &B, N, lut);
}

ORC_API void orc_bumps_truth(const double* mu, const double* amp, const double* width, int K, double base,
                             const double* dirs, int64_t Q, double* out)
{
    bump_ctx B = {mu, amp, width, K, base};
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        double g[3], Rv = 0.0;
        for (int pass = 0; pass < 3; ++pass) {
            hd x[3];
            for (int k = 0; k < 3; ++k) { x[k] = hc(dirs[3 * q + k]); x[k].a = (k == pass) ? 1.0 : 0.0; }
            hd n = hsqrt(hadd(hadd(hmul(x[0], x[0]), hmul(x[1], x[1])), hmul(x[2], x[2])));
            hd in = hinv(n);
            hd R = bump_fn(&B, hmul(x[0], in), hmul(x[1], in), hmul(x[2], in));
            g[pass] = R.a * n.v;
            Rv = R.v;
        }
        out[4 * q] = Rv;
        for (int k = 0; k < 3; ++k) out[4 * q + 1 + k] = g[k];
    }
}

/* ------------------------------------------------------------------------ */
/* General-mode bake (Sec. 3.3, Alg. 1 line 3): central differences in      */
/* (u, v) on the padded grid, using a one-texel bake-time margin.            */
/* ------------------------------------------------------------------------ */

/* Directions of the padded grid with an extra margin ring: index p in
 * 0..N+3 sits at u = (p - 3/2)/N (p = 1..N+2 are the stored texels 0..N+1).
 * dirs = [6][N+4][N+4][3], unit length. */
ORC_API void orc_margin_dirs(int N, double* dirs)
{
    int P = N + 4;
    for (int face = 0; face < 6; ++face)
        for (int q = 0; q < P; ++q)
            for (int p = 0; p < P; ++p) {
                double u = ((double)p - 1.5) / (double)N, v = ((double)q - 1.5) / (double)N;
                double wt[3], n = 0.0;
                for (int k = 0; k < 3; ++k) { wt[k] = FM[face][k] + (2 * u - 1) * FS[face][k] + (2 * v - 1) * FT[face][k]; n += wt[k] * wt[k]; }
                n = sqrt(n);
                double* o = dirs + (((size_t)face * P + q) * P + p) * 3;
                for (int k = 0; k < 3; ++k) o[k] = wt[k] / n;
            }
}

/* samples = [6][N+4][N+4] function values at orc_margin_dirs(N) -> lut.
 * r_u h  = (r[p+1] - r[p-1]) / 2,  r_v h likewise,
 * r_uv h^2 = (r[p+1,q+1] - r[p+1,q-1] - r[p-1,q+1] + r[p-1,q-1]) / 4. */
ORC_API void orc_bake_fd(const double* samples, int N, double* lut)
{
    int P = N + 4;
    for (int face = 0; face < 6; ++face)
        for (int q = 0; q < N + 2; ++q)
            for (int p = 0; p < N + 2; ++p) {
                const double* S = samples + (size_t)face * P * P;
#define SM(pp, qq) S[(size_t)(qq) * P + (pp)]
                int pp = p + 1, qq = q + 1;
                double* o = lut + texel_index(N, face, p, q);
                o[0] = SM(pp, qq);
                o[1] = 0.5 * (SM(pp + 1, qq) - SM(pp - 1, qq));
                o[2] = 0.5 * (SM(pp, qq + 1) - SM(pp, qq - 1));
                o[3] = 0.25 * (SM(pp + 1, qq + 1) - SM(pp + 1, qq - 1) - SM(pp - 1, qq + 1) + SM(pp - 1, qq - 1));
#undef SM
            }
}

/* ------------------------------------------------------------------------ */
/* Backward (differentiation form)                                           */
/* ------------------------------------------------------------------------ */
/* Given upstream g[q] = (gR, g_grad_x, g_grad_y, g_grad_z) of a loss L:
 *  grad_lut: dL/dLUT.  The outputs are linear in the 16 footprint scalars,
 *    so d(out)/d(scalar k) is the forward evaluated on the unit vector e_k;
 *    contributions are summed sequentially in query order.
 *  grad_dirs: dL/dd, forward-mode (hyper-dual e1 part) along each input
 *    axis with face and cell frozen at the input's own.
 * Either output may be NULL.  grad_lut is overwritten. */
ORC_API void orc_backward(const double* lut, int N, const float* dirs, int64_t Q, const double* g, double* grad_lut,
                          double* grad_dirs)
{
    if (grad_lut) {
        size_t T = (size_t)6 * (N + 2) * (N + 2) * 4;
        memset(grad_lut, 0, T * sizeof(double));
        for (int64_t q = 0; q < Q; ++q) {
            double d[3] = {dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2]};
            loc_t L;
            if (!locate(d, N, &L)) continue; /* invalid directions contribute nothing */
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i)
                    for (int ch = 0; ch < 4; ++ch) {
                        double C[2][2][4];
                        memset(C, 0, sizeof C);
                        C[j][i][ch] = 1.0;
                        hd r, ru, rv;
                        reconstruct_hd(C, N, hc(L.s), hc(L.t), &r, &ru, &rv);
                        transport_t Tr;
                        transport_hd(L.face, hc(L.a), hc(L.b), ru, rv, &Tr);
                        double w = g[4 * q] * r.v;
                        for (int k = 0; k < 3; ++k) w += g[4 * q + 1 + k] * Tr.grad[k].v;
                        grad_lut[texel_index(N, L.face, L.i0 + i, L.j0 + j) + ch] += w;
                    }
        }
    }
    if (grad_dirs) {
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < Q; ++q) {
            double d[3] = {dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2]};
            for (int axis = 0; axis < 3; ++axis) {
                double dd[3] = {0.0, 0.0, 0.0};
                dd[axis] = 1.0;
                query_t QR;
                if (!query_hd(lut, N, d, dd, &QR)) { grad_dirs[3 * q + axis] = NAN; continue; }
                double acc = g[4 * q] * QR.R.a;
                for (int k = 0; k < 3; ++k) acc += g[4 * q + 1 + k] * QR.T.grad[k].a;
                grad_dirs[3 * q + axis] = acc;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Bounding radius: Bernstein bound over every cell (convex-hull property)   */
/* ------------------------------------------------------------------------ */
/* 1-D Hermite (p0, m0, p1, m1) on [0,1] -> Bezier (p0, p0+m0/3, p1-m1/3, p1) */
static void herm_to_bez(const double h[4], double b[4])
{
    b[0] = h[0];
    b[1] = h[0] + h[1] / 3.0;
    b[2] = h[2] - h[3] / 3.0;
    b[3] = h[2];
}

/* Bezier control net Bz[a][b] (a along s, b along t) of one cell's bicubic
 * patch: the Hermite data of Eq. (4) converted per direction. */
static void cell_bezier(const double* lut, int N, int face, int i0, int j0, double Bz[4][4])
{
    double C[2][2][4];
    gather_corners(lut, N, face, i0, j0, C);
    /* geometry G[a][b]: a over (p0, m0, p1, m1) in s, b likewise in t */
    double G[4][4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            G[2 * i][2 * j] = C[j][i][0];
            G[2 * i + 1][2 * j] = C[j][i][1];
            G[2 * i][2 * j + 1] = C[j][i][2];
            G[2 * i + 1][2 * j + 1] = C[j][i][3];
        }
    double Hs[4][4];
    for (int b = 0; b < 4; ++b) {
        double col[4] = {G[0][b], G[1][b], G[2][b], G[3][b]}, out[4];
        herm_to_bez(col, out);
        for (int a = 0; a < 4; ++a) Hs[a][b] = out[a];
    }
    for (int a = 0; a < 4; ++a) herm_to_bez(Hs[a], Bz[a]);
}

ORC_API void orc_cell_bezier(const double* lut, int N, int face, int i0, int j0, double* out16)
{
    double Bz[4][4];
    cell_bezier(lut, N, face, i0, j0, Bz);
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) out16[4 * a + b] = Bz[a][b];
}

/* Largest Bezier control point of any cell (absval: largest |control
 * point|, which bounds |r|, the radius of a signed function). */
ORC_API double orc_rmax_bound(const double* lut, int N, int absval)
{
    double best = -INFINITY;
    for (int face = 0; face < 6; ++face)
        for (int j0 = 0; j0 <= N; ++j0)
            for (int i0 = 0; i0 <= N; ++i0) {
                double Bz[4][4];
                cell_bezier(lut, N, face, i0, j0, Bz);
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) {
                        double v = absval ? fabs(Bz[a][b]) : Bz[a][b];
                        if (v > best) best = v;
                    }
            }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Ray casting against the star-shaped surface, Sec. 3.1                     */
/* ------------------------------------------------------------------------ */
/* F(t) = |o + t d - c| - R(w),  F'(t) = d.w - (d . grad R) / |o + t d - c|,
 * d normalised.  Schedule (fixed counts, no early exit after the bracket):
 *   1. bounding sphere |x - c| = rmax -> [t_in, t_out]; miss if none or t_out < 0
 *   2. t0 = max(t_in, 0), t1 = t_out; march t_k = t0 + k (t1 - t0)/K, k = 1..K;
 *      the first k with F(t_k) < 0 brackets [t_{k-1}, t_k]; none -> miss
 *   3. n_bisect halvings of the bracket by the sign of F at the midpoint
 *   4. n_newton safeguarded Newton steps from the bracket midpoint; each step
 *      evaluates F, F' at t, shrinks the bracket by the sign of F(t), and
 *      takes t - F/F' if it lies in the closed bracket, else the bracket
 *      midpoint
 *   5. one last evaluation at the final t gives R, grad R and the normal
 * Outputs: t (+inf for a miss), out4 = (R, grad) and normal3 (NaN on a miss).
 * R is the rendered radius (scale s, optionally signed: R = s |r|). */
typedef struct { double F, dF, R, g[3], w[3]; int ok, sgn; } feval_t;

static feval_t trace_eval(const double* lut, int N, const double o[3], const double c[3], const double dn[3], double t,
                          double scale, int signed_)
{
    feval_t E;
    double p[3];
    for (int k = 0; k < 3; ++k) p[k] = o[k] + t * dn[k] - c[k];
    query_t QR;
    E.ok = query_hd(lut, N, p, NULL, &QR);
    if (!E.ok) { E.F = NAN; E.dF = NAN; E.sgn = 0; return E; }
    double len = sqrt(dot3(p, p)), gr[3];
    for (int k = 0; k < 3; ++k) { gr[k] = QR.T.grad[k].v; E.w[k] = p[k] / len; }
    E.R = rendered(QR.R.v, gr, scale, signed_, E.g, &E.sgn);
    E.F = len - E.R;
    E.dF = dot3(dn, E.w) - dot3(dn, E.g) / len;
    return E;
}

/* Bisection budget of a ray (Sec. 3.1: more refinement for glyphs that
 * project larger, the projected size estimated from the bounding radius and
 * the depth).  The march bracket is at most 2 rmax / n_march long; at the
 * distance |o - c| it spans e = 2 rmax px / (|o - c| n_march) pixels, px
 * being the focal length in pixels.  Bisect until e <= eps_px, at most
 * n_bisect times.  The decision is taken in FP32 in this fixed order
 * (halving is exact), so any implementation of it picks the same count;
 * px <= 0 means the fixed count n_bisect. */
static int bisect_budget(const float o[3], const float c[3], float rmax, float px, float eps_px, int n_march, int n_bisect)
{
    if (!(px > 0.0f)) return n_bisect;
    float ox = o[0] - c[0], oy = o[1] - c[1], oz = o[2] - c[2];
    float dd = ox * ox + oy * oy + oz * oz;
    float depth = sqrtf(dd);
    float e = (2.0f * rmax * px) / (depth * (float)n_march);
    int k = 0;
    while (k < n_bisect && e > eps_px) { e *= 0.5f; ++k; }
    return k;
}

ORC_API int orc_bisect_budget(const float* o, const float* c, float rmax, float px, float eps_px, int n_march, int n_bisect)
{
    return bisect_budget(o, c, rmax, px, eps_px, n_march, n_bisect);
}

/* Full form: scale, signed, adaptive budget (px > 0; the FP32 centre and
 * rmax decide the budget), per-ray sign of r at the hit (0 on a miss) and
 * number of F evaluations.  orc_trace is the plain form. */
ORC_API void orc_trace_ex(const double* lut, int N, const float* center_f, float rmax_f, double scale, int signed_,
                          float px, float eps_px, const float* ray_o, const float* ray_d, int64_t P, int n_march,
                          int n_bisect, int n_newton, double* t_out, double* out4, double* normal3, int8_t* sign,
                          int32_t* evals)
{
    const double center[3] = {center_f[0], center_f[1], center_f[2]}, rmax = rmax_f;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < P; ++r) {
        const int nb = bisect_budget(ray_o + 3 * r, center_f, rmax_f, px, eps_px, n_march, n_bisect);
        int ne = 0;
        double o[3] = {ray_o[3 * r], ray_o[3 * r + 1], ray_o[3 * r + 2]};
        double d[3] = {ray_d[3 * r], ray_d[3 * r + 1], ray_d[3 * r + 2]};
        double dl = sqrt(dot3(d, d));
        double dn[3] = {d[0] / dl, d[1] / dl, d[2] / dl};
        double oc[3] = {o[0] - center[0], o[1] - center[1], o[2] - center[2]};
        double b = dot3(oc, dn), cc = dot3(oc, oc) - rmax * rmax;
        double disc = b * b - cc;
        int hit = 0;
        double t = INFINITY;
        if (disc >= 0.0 && dl > 0.0) {
            double sq = sqrt(disc);
            double tin = -b - sq, tout = -b + sq;
            if (tout >= 0.0) {
                double t0 = tin > 0.0 ? tin : 0.0, t1 = tout;
                double lo = t0, hi = t0;
                for (int k = 1; k <= n_march; ++k) {
                    double tk = t0 + (double)k * (t1 - t0) / (double)n_march;
                    feval_t E = trace_eval(lut, N, o, center, dn, tk, scale, signed_);
                    ++ne;
                    if (E.ok && E.F < 0.0) { hit = 1; lo = t0 + (double)(k - 1) * (t1 - t0) / (double)n_march; hi = tk; break; }
                }
                if (hit) {
                    for (int it = 0; it < nb; ++it) {
                        double mid = 0.5 * (lo + hi);
                        feval_t E = trace_eval(lut, N, o, center, dn, mid, scale, signed_);
                        ++ne;
                        if (E.F < 0.0) hi = mid; else lo = mid;
                    }
                    t = 0.5 * (lo + hi);
                    for (int it = 0; it < n_newton; ++it) {
                        feval_t E = trace_eval(lut, N, o, center, dn, t, scale, signed_);
                        ++ne;
                        if (E.F < 0.0) hi = t; else lo = t;
                        double tn = t - E.F / E.dF;
                        if (!(tn >= lo && tn <= hi)) tn = 0.5 * (lo + hi);
                        t = tn;
                    }
                }
            }
        }
        t_out[r] = hit ? t : INFINITY;
        if (hit) {
            feval_t E = trace_eval(lut, N, o, center, dn, t, scale, signed_);
            ++ne;
            out4[4 * r] = E.R;
            for (int k = 0; k < 3; ++k) out4[4 * r + 1 + k] = E.g[k];
            if (normal3) normal_of(E.R, E.w, E.g, normal3 + 3 * r);
            if (sign) sign[r] = (int8_t)E.sgn;
        } else {
            for (int k = 0; k < 4; ++k) out4[4 * r + k] = NAN;
            if (normal3) for (int k = 0; k < 3; ++k) normal3[3 * r + k] = NAN;
            if (sign) sign[r] = 0;
        }
        if (evals) evals[r] = ne;
    }
}

ORC_API void orc_trace(const double* lut, int N, const double* center, double rmax, const float* ray_o, const float* ray_d,
                       int64_t P, int n_march, int n_bisect, int n_newton, double* t_out, double* out4, double* normal3)
{
    const float c[3] = {(float)center[0], (float)center[1], (float)center[2]};
    orc_trace_ex(lut, N, c, (float)rmax, 1.0, 0, 0.0f, 0.0f, ray_o, ray_d, P, n_march, n_bisect, n_newton, t_out, out4,
                 normal3, NULL, NULL);
}

/* F(t) of one ray at explicit t values (pin tests and hit validation). */
ORC_API void orc_trace_F(const double* lut, int N, const double* center, const double* o, const double* d,
                         const double* ts, int64_t n, double* F)
{
    double dl = sqrt(dot3(d, d));
    double dn[3] = {d[0] / dl, d[1] / dl, d[2] / dl};
    for (int64_t i = 0; i < n; ++i) {
        feval_t E = trace_eval(lut, N, o, center, dn, ts[i], 1.0, 0);
        F[i] = E.F;
    }
}

/* ------------------------------------------------------------------------ */
/* Comparison reconstructions of the paper's experiments (Sec. 4.2, 4.5, 4.6; */
/* Tables psnr_value, cost_extended, runtime) on a value-only LUT.          */
/* ------------------------------------------------------------------------ */
/* Value-only LUT: vlut[face][q][p], p, q in 0..N+3, texel p centred at
 * u = (p - 3/2)/N (a two-texel gutter: the 4x4 bicubic footprint of any
 * cell the faces' queries reach stays inside the table).  Continuous
 * coordinate f = u N + 3/2.
 *   method 0  nearest texel (value only, zero gradient)
 *   method 1  bilinear value; chart derivatives by central differences of the
 *             bilinear reconstruction at u +- h, v +- h (four extra lookups)
 *   method 2  16-tap Catmull-Rom bicubic value and its analytic derivatives
 *   method 3  "fast bicubic" (Table cost_extended): the uniform cubic B-spline
 *             of the samples (the filter a 4-bilinear-fetch evaluation
 *             computes); chart derivatives by the central differences of
 *             method 1, the finite-difference fallback the table lists
 * The chart derivatives become the spherical gradient as in Sec. 3.4. */
static double vl_at(const double* vl, int N, int f, int p, int q)
{
    int P = N + 4;
    if (p < 0) p = 0;
    if (q < 0) q = 0;
    if (p > N + 3) p = N + 3;
    if (q > N + 3) q = N + 3;
    return vl[((size_t)f * P + q) * P + p];
}

static double bilinear_at(const double* vl, int N, int face, double a, double b)
{
    double fu = (a + 1.0) * 0.5 * N + 1.5, fv = (b + 1.0) * 0.5 * N + 1.5;
    int i0 = (int)floor(fu), j0 = (int)floor(fv);
    double s = fu - i0, t = fv - j0;
    return (1 - s) * (1 - t) * vl_at(vl, N, face, i0, j0) + s * (1 - t) * vl_at(vl, N, face, i0 + 1, j0) +
           (1 - s) * t * vl_at(vl, N, face, i0, j0 + 1) + s * t * vl_at(vl, N, face, i0 + 1, j0 + 1);
}

/* Catmull-Rom weights of taps -1, 0, 1, 2 at t, and their derivatives */
static void catmull_rom(double t, double w[4], double dw[4])
{
    double t2 = t * t, t3 = t2 * t;
    w[0] = 0.5 * (-t3 + 2 * t2 - t);
    w[1] = 0.5 * (3 * t3 - 5 * t2 + 2);
    w[2] = 0.5 * (-3 * t3 + 4 * t2 + t);
    w[3] = 0.5 * (t3 - t2);
    dw[0] = 0.5 * (-3 * t2 + 4 * t - 1);
    dw[1] = 0.5 * (9 * t2 - 10 * t);
    dw[2] = 0.5 * (-9 * t2 + 8 * t + 1);
    dw[3] = 0.5 * (3 * t2 - 2 * t);
}

/* uniform cubic B-spline weights of taps -1, 0, 1, 2 at t */
static void bspline3(double t, double w[4])
{
    double t2 = t * t, t3 = t2 * t, m = 1.0 - t;
    w[0] = m * m * m / 6.0;
    w[1] = (3 * t3 - 6 * t2 + 4) / 6.0;
    w[2] = (-3 * t3 + 3 * t2 + 3 * t + 1) / 6.0;
    w[3] = t3 / 6.0;
}

ORC_API void orc_baseline_query(const double* vlut, int N, const float* dirs, int64_t Q, int method, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        double d[3] = {dirs[3 * q], dirs[3 * q + 1], dirs[3 * q + 2]};
        int f = face_select(d[0], d[1], d[2]);
        if (f < 0) { for (int k = 0; k < 4; ++k) out[4 * q + k] = NAN; continue; }
        double a = dot3(d, FS[f]) / dot3(d, FM[f]), b = dot3(d, FT[f]) / dot3(d, FM[f]);
        double fu = (a + 1.0) * 0.5 * N + 1.5, fv = (b + 1.0) * 0.5 * N + 1.5;
        double R = 0, ru = 0, rv = 0;
        if (method == 0) {
            R = vl_at(vlut, N, f, (int)floor(fu + 0.5), (int)floor(fv + 0.5));
        } else if (method == 1 || method == 3) {
            double h = 1.0 / N, da = 2.0 * h; /* a = 2u - 1: a step of h in u is 2h in a */
            if (method == 1) {
                R = bilinear_at(vlut, N, f, a, b);
            } else {
                int i0 = (int)floor(fu), j0 = (int)floor(fv);
                double ws[4], wt[4];
                bspline3(fu - i0, ws);
                bspline3(fv - j0, wt);
                for (int j = 0; j < 4; ++j)
                    for (int i = 0; i < 4; ++i) R += ws[i] * wt[j] * vl_at(vlut, N, f, i0 - 1 + i, j0 - 1 + j);
            }
            ru = (bilinear_at(vlut, N, f, a + da, b) - bilinear_at(vlut, N, f, a - da, b)) / (2 * h);
            rv = (bilinear_at(vlut, N, f, a, b + da) - bilinear_at(vlut, N, f, a, b - da)) / (2 * h);
        } else {
            int i0 = (int)floor(fu), j0 = (int)floor(fv);
            double s = fu - i0, t = fv - j0, ws[4], dws[4], wt[4], dwt[4];
            catmull_rom(s, ws, dws);
            catmull_rom(t, wt, dwt);
            for (int j = 0; j < 4; ++j)
                for (int i = 0; i < 4; ++i) {
                    double v = vl_at(vlut, N, f, i0 - 1 + i, j0 - 1 + j);
                    R += ws[i] * wt[j] * v;
                    ru += dws[i] * wt[j] * v;
                    rv += ws[i] * dwt[j] * v;
                }
            ru *= N;
            rv *= N;
        }
        double g[3];
        transport_closed(f, a, b, ru, rv, g);
        out[4 * q] = R;
        for (int k = 0; k < 3; ++k) out[4 * q + 1 + k] = g[k];
    }
}

/* ------------------------------------------------------------------------ */
/* Mip chain (Sec. 4.7, Table lod)                                           */
/* ------------------------------------------------------------------------ */
/* Next level of a TEXEL LUT of face size N (even) -> N/2.
 * Consistent (mode 0): the value field is box-filtered -- the coarse value at
 *   a texel centre is the mean of the fine map at the four fine texel-centre
 *   directions the coarse texel covers (evaluated as queries, so points
 *   outside the face read the neighbouring face) -- on the coarse padded grid
 *   plus a margin ring, and the derivative channels are recomputed from the
 *   filtered values by central differences (the general-mode bake).
 * Naive (mode 1): as consistent, but every interior coarse texel holds the
 *   plain average of the four fine texels' stored channels
 *   (r, r_u h, r_v h, r_uv h^2), as a box-filtering mip generator would. */
ORC_API void orc_mip_level(const double* lut, int N, int mode, double* out)
{
    int Nc = N / 2, Pm = Nc + 4, P = N + 2;
    double* samples = (double*)malloc(sizeof(double) * 6 * Pm * Pm);
#pragma omp parallel for collapse(2) schedule(static)
    for (int face = 0; face < 6; ++face)
        for (int q = 0; q < Pm; ++q)
            for (int p = 0; p < Pm; ++p) {
                /* coarse texel (p, q) of the margin grid: u = (p - 3/2)/Nc; its
                 * fine sub-texel centres sit at u -+ 1/(2N) */
                double uc = ((double)p - 1.5) / Nc, vc = ((double)q - 1.5) / Nc, acc = 0.0;
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a) {
                        double u = uc + (a ? 0.5 : -0.5) / N, v = vc + (b ? 0.5 : -0.5) / N;
                        double d[3];
                        for (int k = 0; k < 3; ++k) d[k] = FM[face][k] + (2 * u - 1) * FS[face][k] + (2 * v - 1) * FT[face][k];
                        query_t QR;
                        query_hd(lut, N, d, NULL, &QR);
                        acc += QR.R.v;
                    }
                samples[((size_t)face * Pm + q) * Pm + p] = 0.25 * acc;
            }
    orc_bake_fd(samples, Nc, out);
    free(samples);
    if (mode == 1) {
        for (int face = 0; face < 6; ++face)
            for (int q = 1; q <= Nc; ++q)
                for (int p = 1; p <= Nc; ++p)
                    for (int ch = 0; ch < 4; ++ch) {
                        double acc = 0.0;
                        for (int b = 0; b < 2; ++b)
                            for (int a = 0; a < 2; ++a)
                                acc += lut[(((size_t)face * P + (2 * q - 1 + b)) * P + (2 * p - 1 + a)) * 4 + ch];
                        out[texel_index(Nc, face, p, q) + ch] = 0.25 * acc;
                    }
    }
}

ORC_API int orc_version(void) { return 1; }

#ifdef _OPENMP
#include <omp.h>
ORC_API int orc_num_threads(void) { return omp_get_max_threads(); }
ORC_API void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
#else
ORC_API int orc_num_threads(void) { return 1; }
ORC_API void orc_set_threads(int n) { (void)n; }
#endif

/* ------------------------------------------------------------------------ */
/* Radial depth of a triangle mesh (Sec. 4.9, mesh LOD impostors)            */
/* ------------------------------------------------------------------------ */
/* R(w) = max{t >= 0 : c + t w lies on the mesh surface}: the farthest
 * intersection of the ray from the centre c along the unit direction w with
 * any triangle (closed triangles; 0 when the ray meets none).  Every
 * triangle is tested (no acceleration structure), by solving
 * c + t w = v0 + a (v1 - v0) + b (v2 - v0) with Cramer's rule and keeping
 * a >= 0, b >= 0, a + b <= 1 (each with a 1e-12 tolerance, so that a ray
 * through a shared edge or vertex meets the triangles around it).
 * Triangles with an index outside [0, V) are skipped. */
ORC_API void orc_mesh_radial_depth(const double* verts, int64_t V, const int32_t* tris, int64_t T, const double* c,
                                   const float* dirs, int64_t P, double* depth)
{
    const double tol = 1e-12;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < P; ++r) {
        double w[3] = {dirs[3 * r], dirs[3 * r + 1], dirs[3 * r + 2]};
        double n = sqrt(dot3(w, w));
        double best = 0.0;
        if (n > 0.0 && isfinite(n)) {
            for (int k = 0; k < 3; ++k) w[k] /= n;
            for (int64_t f = 0; f < T; ++f) {
                int64_t i0 = tris[3 * f], i1 = tris[3 * f + 1], i2 = tris[3 * f + 2];
                if (i0 < 0 || i0 >= V || i1 < 0 || i1 >= V || i2 < 0 || i2 >= V) continue;
                double e1[3], e2[3], s[3];
                for (int k = 0; k < 3; ++k) {
                    e1[k] = verts[3 * i1 + k] - verts[3 * i0 + k];
                    e2[k] = verts[3 * i2 + k] - verts[3 * i0 + k];
                    s[k] = c[k] - verts[3 * i0 + k];
                }
                /* [-w e1 e2] (t a b)^T = s */
                double m[3][3];
                for (int k = 0; k < 3; ++k) { m[k][0] = -w[k]; m[k][1] = e1[k]; m[k][2] = e2[k]; }
                double det = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
                             m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
                             m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
                if (det == 0.0) continue; /* ray parallel to the triangle's plane */
                double x[3];
                for (int col = 0; col < 3; ++col) {
                    double a[3][3];
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) a[i][j] = (j == col) ? s[i] : m[i][j];
                    double dc = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                                a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                                a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
                    x[col] = dc / det;
                }
                double t = x[0], a = x[1], b = x[2];
                if (a >= -tol && b >= -tol && a + b <= 1.0 + tol && t >= 0.0 && t > best) best = t;
            }
        }
        depth[r] = best;
    }
}
