"""Pins for the FP64 oracle: checks against what the paper and the
mathematics fix, independent of the oracle's own code paths.

Each test names the passage it pins.  None of them re-types an oracle
formula and compares it with itself: the expected values come from hand
worked tables (golden files), closed forms, polynomial reproduction,
finite differences, invariants, exact adjoints or convergence orders.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from conftest import load_golden

# Test-side cube-map table, typed from the published selection table (the
# golden file cubemap_faces.txt pins it): d/|ma| = M + sc S + tc T.
TM = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
TS = np.array([[0, 0, -1], [0, 0, 1], [1, 0, 0], [1, 0, 0], [1, 0, 0], [-1, 0, 0]], float)
TT = np.array([[0, -1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1], [0, -1, 0], [0, -1, 0]], float)


def chart_dir(face, u, v):
    """Unit direction of chart point (u, v) of a face (extended plane)."""
    u = np.asarray(u, float)
    v = np.asarray(v, float)
    w = TM[face] + (2 * u - 1)[..., None] * TS[face] + (2 * v - 1)[..., None] * TT[face]
    return w / np.linalg.norm(w, axis=-1, keepdims=True)


def face_uv(d):
    """(face, u, v) of directions by the published table (test-side)."""
    d = np.asarray(d, float)
    ax, ay, az = np.abs(d).T
    face = np.where((ax >= ay) & (ax >= az), np.where(d[:, 0] >= 0, 0, 1),
                    np.where(ay >= az, np.where(d[:, 1] >= 0, 2, 3), np.where(d[:, 2] >= 0, 4, 5)))
    ma = np.einsum("ij,ij->i", d, TM[face])
    sc = np.einsum("ij,ij->i", d, TS[face])
    tc = np.einsum("ij,ij->i", d, TT[face])
    return face, 0.5 * (sc / ma + 1), 0.5 * (tc / ma + 1)


def rng(k=0):
    return np.random.default_rng(1234 + k)


# ---------------------------------------------------------------------------
# Hermite basis, Sec. 3.3 Eq. (3)
# ---------------------------------------------------------------------------
def test_hermite_cardinal_conditions():
    b0 = oracle.hermite_basis(0.0)
    b1 = oracle.hermite_basis(1.0)
    # values H0, H1, H0d, H1d at s=0 and s=1
    assert list(b0[:4]) == [1.0, 0.0, 0.0, 0.0]
    assert list(b1[:4]) == [0.0, 1.0, 0.0, 0.0]
    # derivatives H0', H1', H0d', H1d'
    assert list(b0[4:]) == [0.0, 0.0, 1.0, 0.0]
    assert list(b1[4:]) == [0.0, 0.0, 0.0, 1.0]


def test_hermite_partition_and_derivative_consistency():
    for s in rng().uniform(-0.5, 1.5, 50):
        b = oracle.hermite_basis(s)
        assert abs(b[0] + b[1] - 1.0) < 1e-14
        h = 1e-6
        fd = (oracle.hermite_basis(s + h)[:4] - oracle.hermite_basis(s - h)[:4]) / (2 * h)
        np.testing.assert_allclose(b[4:], fd, atol=1e-8)


# ---------------------------------------------------------------------------
# Cube-map mapping, Sec. 3.2
# ---------------------------------------------------------------------------
def test_cubemap_golden_table():
    rows = load_golden("cubemap_faces.txt")
    N = 16
    for x, y, z, face, u, v in rows:
        f, i0, j0, s, t = oracle.locate(np.array([[x, y, z]], np.float32), N)
        assert f[0] == int(face), (x, y, z)
        assert abs((i0[0] + s[0] - 0.5) / N - u) < 1e-12, (x, y, z)
        assert abs((j0[0] + t[0] - 0.5) / N - v) < 1e-12, (x, y, z)


def test_test_table_matches_golden():
    rows = np.array(load_golden("cubemap_faces.txt"))
    f, u, v = face_uv(rows[:, :3])
    np.testing.assert_array_equal(f, rows[:, 3].astype(int))
    np.testing.assert_allclose(u, rows[:, 4], atol=1e-15)
    np.testing.assert_allclose(v, rows[:, 5], atol=1e-15)


def test_locate_fp64_decision_and_local_coords():
    """Cell = floor of the FP64 coordinate f = u N + 1/2 (texel p centred at
    u = (p - 1/2)/N, Sec. 3.2), u from this test's own face table."""
    d = workloads.uniform_dirs(20000, rng(1))
    for N in (10, 32, 257):
        f, i0, j0, s, t = oracle.locate(d, N)
        ff, uu, vv = face_uv(d.astype(np.float64))
        np.testing.assert_array_equal(f, ff)
        fu, fv = uu * N + 0.5, vv * N + 0.5
        # away from cell edges (where FP64 rounding of the two routes could
        # differ) the cell is floor(f)
        far = (np.abs(fu - np.round(fu)) > 1e-12) & (np.abs(fv - np.round(fv)) > 1e-12)
        assert far.mean() > 0.999
        np.testing.assert_array_equal(i0[far], np.minimum(np.floor(fu[far]), N).astype(np.int32))
        np.testing.assert_array_equal(j0[far], np.minimum(np.floor(fv[far]), N).astype(np.int32))
        # the FP64 local coordinate agrees with the test-side u
        np.testing.assert_allclose(i0 + s, uu * N + 0.5, atol=1e-9)
        np.testing.assert_allclose(j0 + t, vv * N + 0.5, atol=1e-9)
        assert s.min() > -1e-5 and s.max() < 1 + 1e-5
        assert i0.min() >= 0 and i0.max() <= N


def test_invalid_directions_give_nan():
    lut = workloads.random_lut(8, rng(2))
    d = np.array([[0, 0, 0], [np.nan, 1, 0], [np.inf, 0, 0], [1, 0, 0]], np.float32)
    out = oracle.query(lut, d)
    assert np.all(np.isnan(out[:3]))
    assert np.all(np.isfinite(out[3]))


# ---------------------------------------------------------------------------
# Reconstruction, Sec. 3.3 Eqs. (4)-(5)
# ---------------------------------------------------------------------------
def poly_lut(N, C):
    """LUT holding (P, P_u h, P_v h, P_uv h^2) of per-face bicubics
    P_f(u,v) = sum_ab C[f,a,b] u^a v^b at the texel centres u_p=(p-1/2)/N."""
    p = (np.arange(N + 2) - 0.5) / N
    U, V = np.meshgrid(p, p, indexing="xy")  # [q, p]
    lut = np.zeros((6, N + 2, N + 2, 4))
    for f in range(6):
        P, Pu, Pv, Puv = poly_eval(C[f], U, V)
        lut[f, ..., 0] = P
        lut[f, ..., 1] = Pu / N
        lut[f, ..., 2] = Pv / N
        lut[f, ..., 3] = Puv / N ** 2
    return lut


def poly_eval(c, u, v):
    P = Pu = Pv = Puv = 0.0
    for a in range(4):
        for b in range(4):
            P = P + c[a, b] * u ** a * v ** b
            if a:
                Pu = Pu + c[a, b] * a * u ** (a - 1) * v ** b
            if b:
                Pv = Pv + c[a, b] * b * u ** a * v ** (b - 1)
            if a and b:
                Puv = Puv + c[a, b] * a * b * u ** (a - 1) * v ** (b - 1)
    return P, Pu, Pv, Puv


@pytest.mark.parametrize("N", [4, 10, 33])
def test_reproduces_bicubic_polynomials(N):
    r = rng(N)
    C = r.standard_normal((6, 4, 4))
    lut = poly_lut(N, C)
    d = workloads.uniform_dirs(6000, r)
    ch = oracle.query_chart(lut, d)
    f, u, v = face_uv(d.astype(np.float64))
    for face in range(6):
        m = f == face
        P, Pu, Pv, _ = poly_eval(C[face], u[m], v[m])
        scale = np.abs(C[face]).sum() * 10
        np.testing.assert_allclose(ch[m, 0], P, atol=1e-12 * scale)
        np.testing.assert_allclose(ch[m, 1], Pu, atol=1e-11 * scale)
        np.testing.assert_allclose(ch[m, 2], Pv, atol=1e-11 * scale)


def test_stored_values_at_texel_centres():
    N = 9
    lut = workloads.random_lut(N, rng(3)).astype(np.float64)
    for face in range(6):
        for i0 in range(N + 1):
            for j0 in (0, 3, N):
                for (i, j) in ((0, 0), (1, 0), (0, 1), (1, 1)):
                    r, ru, rv = oracle.reconstruct(lut, face, i0, j0, float(i), float(j))
                    tex = lut[face, j0 + j, i0 + i]
                    assert r == tex[0]
                    assert abs(ru - N * tex[1]) <= 1e-14 * N
                    assert abs(rv - N * tex[2]) <= 1e-14 * N


def test_c1_across_cell_edges():
    N = 12
    lut = workloads.random_lut(N, rng(4)).astype(np.float64)
    r = rng(5)
    for _ in range(200):
        face = int(r.integers(6))
        i0 = int(r.integers(N))
        j0 = int(r.integers(N + 1))
        t = float(r.uniform())
        a = oracle.reconstruct(lut, face, i0, j0, 1.0, t)
        b = oracle.reconstruct(lut, face, i0 + 1, j0, 0.0, t)
        np.testing.assert_allclose(a, b, atol=1e-13 * N)
        j0 = int(r.integers(N))
        i0 = int(r.integers(N + 1))
        s = float(r.uniform())
        a = oracle.reconstruct(lut, face, i0, j0, s, 1.0)
        b = oracle.reconstruct(lut, face, i0, j0 + 1, s, 0.0)
        np.testing.assert_allclose(a, b, atol=1e-13 * N)


# ---------------------------------------------------------------------------
# Gradient transport, Sec. 3.4 Eqs. (6)-(9), and the normal, Eq. (10)
# ---------------------------------------------------------------------------
def test_transport_identities():
    N = 16
    lut = workloads.random_lut(N, rng(6))
    d = workloads.uniform_dirs(5000, rng(7))
    out = oracle.query(lut, d)
    closed = oracle.query(lut, d, closed_form=True)
    scale = np.linalg.norm(out[:, 1:], axis=1).max()
    np.testing.assert_allclose(out, closed, atol=1e-12 * scale)
    ch = oracle.query_chart(lut, d)
    a, b = ch[:, 5], ch[:, 6]
    rho2 = 1 + a * a + b * b
    np.testing.assert_allclose(ch[:, 3], 16.0 / rho2 ** 3, rtol=1e-12)  # det G = 16 / rho^6
    assert ch[:, 3].min() >= 16.0 / 27.0 - 1e-12  # clamp is inert on a face
    assert np.all(ch[:, 4] == 0)
    w = ch[:, 7:10]
    g = out[:, 1:]
    assert np.abs(np.einsum("ij,ij->i", g, w)).max() < 1e-12 * scale
    # grad . e1 = r_u, grad . e2 = r_v with e1, e2 from finite differences of
    # the test-side chart map
    f, u, v = face_uv(d.astype(np.float64))
    h = 1e-6
    e1 = np.stack([(chart_dir(ff, uu + h, vv) - chart_dir(ff, uu - h, vv)) / (2 * h) for ff, uu, vv in zip(f, u, v)])
    e2 = np.stack([(chart_dir(ff, uu, vv + h) - chart_dir(ff, uu, vv - h)) / (2 * h) for ff, uu, vv in zip(f, u, v)])
    np.testing.assert_allclose(np.einsum("ij,ij->i", g, e1), ch[:, 1], atol=1e-7 * scale)
    np.testing.assert_allclose(np.einsum("ij,ij->i", g, e2), ch[:, 2], atol=1e-7 * scale)


def test_gradient_matches_fd_of_reconstruction():
    """The spherical gradient equals central differences of the reconstructed
    value along tangent directions (catches a wrong sign, index or
    transposed operand anywhere in Eqs. (5)-(9))."""
    N = 8
    c = workloads.sh_glyph_coeffs(6, 1, rng(8))[0]
    lut = oracle.bake_sh(c, N)
    d = workloads.uniform_dirs(3000, rng(9)).astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    f, i0, j0, s, t = oracle.locate(d.astype(np.float32), N)
    keep = (s > 0.05) & (s < 0.95) & (t > 0.05) & (t < 0.95)
    d = d[keep]
    base = oracle.query_f64(lut, d)
    r = rng(10)
    tau = r.standard_normal(d.shape)
    tau -= np.einsum("ij,ij->i", tau, d)[:, None] * d
    tau /= np.linalg.norm(tau, axis=1, keepdims=True)
    delta = 1e-5 / N
    # geodesic steps w(+-delta) = cos(delta) w +- sin(delta) tau
    dp = math.cos(delta) * d + math.sin(delta) * tau
    dm = math.cos(delta) * d - math.sin(delta) * tau
    fd = (oracle.query_f64(lut, dp)[:, 0] - oracle.query_f64(lut, dm)[:, 0]) / (2 * delta)
    an = np.einsum("ij,ij->i", base[:, 1:], tau)
    scale = np.linalg.norm(base[:, 1:], axis=1).max()
    assert np.abs(fd - an).max() < 1e-6 * scale


def test_constant_lut_gives_sphere():
    N = 7
    lut = np.zeros((6, N + 2, N + 2, 4))
    lut[..., 0] = 1.25
    d = workloads.uniform_dirs(2000, rng(11))
    out, n = oracle.query(lut, d, normals=True)
    # partition of unity holds up to rounding of the 16-term sum
    assert np.abs(out[:, 0] - 1.25).max() < 1e-15
    assert np.abs(out[:, 1:]).max() < 1e-13
    w = d.astype(np.float64) / np.linalg.norm(d.astype(np.float64), axis=1, keepdims=True)
    np.testing.assert_allclose(n, w, atol=1e-13)


def test_normal_is_gradient_of_implicit_function():
    """n of Eq. (10) is parallel to grad F for F(x) = |x| - R(x/|x|): check
    against central differences of F built from FP64 reconstructions."""
    N = 12
    c = workloads.sh_glyph_coeffs(4, 1, rng(12))[0]
    lut = oracle.bake_sh(c, N)
    d = workloads.uniform_dirs(400, rng(13)).astype(np.float64)
    out, n = oracle.query(lut, d.astype(np.float32), normals=True)
    w = d / np.linalg.norm(d, axis=1, keepdims=True)
    x = w * out[:, :1]  # surface point (centre at origin)
    h = 1e-6
    gF = np.zeros_like(x)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        Fp = np.linalg.norm(x + e, axis=1) - oracle.query_f64(lut, x + e)[:, 0]
        Fm = np.linalg.norm(x - e, axis=1) - oracle.query_f64(lut, x - e)[:, 0]
        gF[:, k] = (Fp - Fm) / (2 * h)
    gF /= np.linalg.norm(gF, axis=1, keepdims=True)
    # compare where the query direction's cell is the same for x +- h
    err = np.linalg.norm(gF - n, axis=1)
    assert np.median(err) < 1e-7
    assert np.mean(err < 1e-6) > 0.97


# ---------------------------------------------------------------------------
# Real spherical harmonics (bake input function)
# ---------------------------------------------------------------------------
def test_sh_closed_forms_low_order():
    d = workloads.uniform_dirs(500, rng(14)).astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    x, y, z = d.T
    Y = oracle.sh_basis(2, d)
    pi = math.pi
    exp = np.stack([
        np.full_like(x, 0.5 / math.sqrt(pi)),
        math.sqrt(3 / (4 * pi)) * y, math.sqrt(3 / (4 * pi)) * z, math.sqrt(3 / (4 * pi)) * x,
        0.5 * math.sqrt(15 / pi) * x * y, 0.5 * math.sqrt(15 / pi) * y * z,
        0.25 * math.sqrt(5 / pi) * (3 * z * z - 1), 0.5 * math.sqrt(15 / pi) * x * z,
        0.25 * math.sqrt(15 / pi) * (x * x - y * y)], axis=1)
    np.testing.assert_allclose(Y, exp, atol=1e-14)


def test_sh_addition_theorem():
    d = workloads.uniform_dirs(300, rng(15)).astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = oracle.sh_basis(16, d)
    for l in range(17):
        s = (Y[:, l * l:(l + 1) * (l + 1)] ** 2).sum(axis=1)
        np.testing.assert_allclose(s, (2 * l + 1) / (4 * math.pi), rtol=1e-11)


@pytest.mark.parametrize("L", [8, 16])
def test_sh_orthonormality_by_quadrature(L):
    nz = L + 1
    zs, wz = np.polynomial.legendre.leggauss(nz)
    nphi = 2 * L + 2
    phi = 2 * math.pi * np.arange(nphi) / nphi
    Z, PHI = np.meshgrid(zs, phi, indexing="ij")
    W = np.repeat(wz, nphi) * (2 * math.pi / nphi)
    sx = np.sqrt(1 - Z ** 2)
    d = np.stack([sx * np.cos(PHI), sx * np.sin(PHI), Z], axis=-1).reshape(-1, 3)
    Y = oracle.sh_basis(L, d)
    G = (Y * W[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye((L + 1) ** 2), atol=1e-12 if L <= 8 else 1e-10)


# ---------------------------------------------------------------------------
# Bake, Sec. 3.3 Alg. 1 (analytic SH mode)
# ---------------------------------------------------------------------------
def test_bake_channels_vs_finite_differences():
    N = 16
    c = workloads.sh_glyph_coeffs(8, 1, rng(16))[0]
    r = rng(17)
    h = 1e-4
    for _ in range(40):
        face = int(r.integers(6))
        u, v = r.uniform(-0.05, 1.05, 2)
        ch = oracle.bake_sh_point(c, N, face, u, v)

        def G(uu, vv):
            return oracle.sh_truth(c, chart_dir(face, np.array([uu]), np.array([vv])))[0, 0]

        g0 = G(u, v)
        gu = (G(u + h, v) - G(u - h, v)) / (2 * h)
        gv = (G(u, v + h) - G(u, v - h)) / (2 * h)
        guv = (G(u + h, v + h) - G(u + h, v - h) - G(u - h, v + h) + G(u - h, v - h)) / (4 * h * h)
        assert abs(ch[0] - g0) < 1e-14
        assert abs(ch[1] - gu / N) < 1e-8
        assert abs(ch[2] - gv / N) < 1e-8
        assert abs(ch[3] - guv / N ** 2) < 1e-7


def test_bake_linear_function_closed_form():
    """R(w) = a . w (degree 1): G(A,B) = (alpha + beta A + gamma B)/sqrt(1+A^2+B^2)
    with A = 2u-1, B = 2v-1, alpha = a.M, beta = a.S, gamma = a.T."""
    avec = np.array([0.3, -0.7, 0.45])
    k = math.sqrt(4 * math.pi / 3)
    c = np.zeros(4)
    c[1], c[2], c[3] = avec[1] * k, avec[2] * k, avec[0] * k  # Y_{1,-1} ~ y, Y_10 ~ z, Y_11 ~ x
    N = 6
    lut = oracle.bake_sh(c, N)
    for face in range(6):
        al, be, ga = avec @ TM[face], avec @ TS[face], avec @ TT[face]
        for q in range(N + 2):
            for p in range(N + 2):
                A = 2 * (p - 0.5) / N - 1
                B = 2 * (q - 0.5) / N - 1
                n = 1 + A * A + B * B
                num = al + be * A + ga * B
                G = num * n ** -0.5
                GA = be * n ** -0.5 - num * A * n ** -1.5
                GB = ga * n ** -0.5 - num * B * n ** -1.5
                GAB = -be * B * n ** -1.5 - ga * A * n ** -1.5 + 3 * num * A * B * n ** -2.5
                exp = [G, 2 * GA / N, 2 * GB / N, 4 * GAB / N ** 2]
                np.testing.assert_allclose(lut[face, q, p], exp, atol=1e-14)


def test_gutter_is_function_at_texel_centre_direction():
    """Sec. 3.2: gutter texels hold the function at their own texel-centre
    direction (on the extended face plane), not a copy of a neighbour."""
    N = 10
    c = workloads.sh_glyph_coeffs(6, 1, rng(18))[0]
    lut = oracle.bake_sh(c, N)
    for face in range(6):
        for (p, q) in ((0, 0), (0, 5), (N + 1, 3), (4, N + 1), (N + 1, N + 1)):
            w = chart_dir(face, np.array([(p - 0.5) / N]), np.array([(q - 0.5) / N]))
            assert abs(lut[face, q, p, 0] - oracle.sh_truth(c, w)[0, 0]) < 1e-14


# ---------------------------------------------------------------------------
# Method vs truth (convergence trend, paper Sec. 4.2 Table psnr_value)
# ---------------------------------------------------------------------------
def test_convergence_orders_and_psnr_trend():
    c = workloads.sh_glyph_coeffs(8, 1, rng(19))[0]
    d = workloads.uniform_dirs(20000, rng(20))
    truth = oracle.sh_truth(c, d.astype(np.float64))
    ev, eg, psnr = [], [], []
    Ns = (8, 16, 32, 64)
    peak = truth[:, 0].max() - truth[:, 0].min()
    for N in Ns:
        out = oracle.query(oracle.bake_sh(c, N), d)
        dv = out[:, 0] - truth[:, 0]
        ev.append(np.sqrt(np.mean(dv ** 2)))
        eg.append(np.sqrt(np.mean(np.sum((out[:, 1:] - truth[:, 1:]) ** 2, axis=1))))
        psnr.append(20 * math.log10(peak / ev[-1]))
    sv = [math.log2(ev[i] / ev[i + 1]) for i in range(3)]
    sg = [math.log2(eg[i] / eg[i + 1]) for i in range(3)]
    # bicubic Hermite with exact derivatives: value O(h^4), gradient O(h^3)
    assert 3.3 < sv[-1] < 5.5, sv
    assert 2.3 < sg[-1] < 4.5, sg
    # Table psnr_value: Hermite gains ~30 dB per doubling from N=8 to 32
    paper = {int(r[0]): r[3] for r in load_golden("psnr_value_table.txt")}
    assert psnr[1] - psnr[0] > 20 and psnr[2] - psnr[1] > 20
    assert (paper[16] - paper[8]) > 20 and (paper[32] - paper[16]) > 20


def test_face_seam_jump_converges():
    """Across a face seam the two faces' patches agree to interpolation
    order (value O(h^4), gradient O(h^3)); no exact equality is claimed."""
    c = workloads.sh_glyph_coeffs(8, 1, rng(21))[0]
    r = rng(22)
    # points on the +X / +Y seam: x = y > |z|
    zz = r.uniform(-0.9, 0.9, 400)
    d = np.stack([np.ones_like(zz), np.ones_like(zz), zz], axis=1)
    jv, jg = [], []
    for N in (16, 32, 64):
        lut = oracle.bake_sh(c, N)
        a = oracle.query_f64(lut, d, face=0)
        b = oracle.query_f64(lut, d, face=2)
        jv.append(np.abs(a[:, 0] - b[:, 0]).max())
        jg.append(np.linalg.norm(a[:, 1:] - b[:, 1:], axis=1).max())
    ov = math.log2(jv[1] / jv[2])
    og = math.log2(jg[1] / jg[2])
    assert ov > 3.5, (jv, ov)
    assert og > 2.5, (jg, og)


# ---------------------------------------------------------------------------
# General-mode (finite difference) bake, Sec. 3.3 Alg. 1
# ---------------------------------------------------------------------------
def test_fd_bake_second_order():
    c = workloads.sh_glyph_coeffs(6, 1, rng(23))[0]
    errs = []
    for N in (16, 32, 64):
        dirs = oracle.margin_dirs(N)
        samples = oracle.sh_truth(c, dirs.reshape(-1, 3))[:, 0].reshape(6, N + 4, N + 4)
        fd = oracle.bake_fd(samples, N)
        an = oracle.bake_sh(c, N)
        np.testing.assert_allclose(fd[..., 0], an[..., 0], atol=1e-14)
        # scaled channels r_u h: FD error O(h^2) relative to r_u, i.e. O(h^3) on r_u h
        errs.append(np.abs(fd[..., 1:3] - an[..., 1:3]).max() * N)
    o = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 1.6 < o[-1] < 2.5, (errs, o)


# ---------------------------------------------------------------------------
# Bounding radius and ray casting, Sec. 3.1
# ---------------------------------------------------------------------------
def test_rmax_bound_is_upper_bound():
    N = 12
    c = workloads.sh_glyph_coeffs(8, 1, rng(24))[0]
    lut = oracle.bake_sh(c, N)
    bound = oracle.rmax_bound(lut)
    d = workloads.uniform_dirs(200000, rng(25))
    m = oracle.query(lut, d)[:, 0].max()
    assert bound >= m
    assert bound < m * 1.05
    lut0 = np.zeros((6, N + 2, N + 2, 4))
    lut0[..., 0] = 0.8
    assert oracle.rmax_bound(lut0) == 0.8


def test_bezier_net_reproduces_patch():
    """The control net behind the bound is the patch in Bernstein form:
    sum_ab B_a(s) B_b(t) Bz[a,b] equals the Hermite reconstruction."""
    N = 7
    lut = workloads.random_lut(N, rng(40)).astype(np.float64)
    r = rng(41)

    def bern(x):
        return np.array([(1 - x) ** 3, 3 * x * (1 - x) ** 2, 3 * x * x * (1 - x), x ** 3])

    for _ in range(100):
        face, i0, j0 = int(r.integers(6)), int(r.integers(N + 1)), int(r.integers(N + 1))
        s, t = r.uniform(0, 1, 2)
        Bz = oracle.cell_bezier(lut, face, i0, j0)
        val = bern(s) @ Bz @ bern(t)
        assert abs(val - oracle.reconstruct(lut, face, i0, j0, s, t)[0]) < 1e-13


def test_trace_constant_sphere_closed_form():
    N = 6
    R0 = 0.9
    lut = np.zeros((6, N + 2, N + 2, 4))
    lut[..., 0] = R0
    r = rng(26)
    P = 500
    o = np.tile(np.array([[0.2, -0.1, 3.0]]), (P, 1))
    tgt = r.uniform(-0.6, 0.6, (P, 3)) * np.array([1, 1, 0])
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o32, d32 = o.astype(np.float32), d.astype(np.float32)
    t, out, n = oracle.trace(lut, np.zeros(3), R0 * 1.05, o32, d32)
    oo = o32.astype(np.float64)
    dd = d32.astype(np.float64)
    dd /= np.linalg.norm(dd, axis=1, keepdims=True)
    b = np.einsum("ij,ij->i", oo, dd)
    cc = np.einsum("ij,ij->i", oo, oo) - R0 * R0
    t_exact = -b - np.sqrt(b * b - cc)
    hit = np.isfinite(t)
    assert hit.all()
    np.testing.assert_allclose(t, t_exact, rtol=1e-12)
    x = oo + t[:, None] * dd
    np.testing.assert_allclose(n, x / np.linalg.norm(x, axis=1, keepdims=True), atol=1e-10)


def z_lut(N):
    """r(w) = z = sqrt(4 pi / 3) Y_1^0 baked analytically: a signed function
    whose rendered radius s|z| is two spheres of radius s/2 centred at
    (0, 0, +-s/2) (|x - c|^2 = s^2 z^2 - s^2 z^2 + s^2/4 on x = s|z| w)."""
    c = np.zeros(4)
    c[2] = math.sqrt(4 * math.pi / 3)
    return oracle.bake_sh(c, N)


def test_signed_radius_two_spheres_closed_form():
    N, s = 48, 0.5
    lut = z_lut(N)
    d = workloads.uniform_dirs(3000, rng(80)).astype(np.float64)
    d = d[np.abs(d[:, 2]) > 0.2]  # away from the kink at z = 0
    out, n, sg = oracle.query_scaled(lut, d, scale=s, signed=True)
    w = d / np.linalg.norm(d, axis=1, keepdims=True)
    z = w[:, 2]
    np.testing.assert_allclose(out[:, 0], s * np.abs(z), atol=1e-7)
    assert np.array_equal(sg, np.sign(z).astype(np.int8))
    x = out[:, :1] * w
    cen = np.zeros_like(x)
    cen[:, 2] = np.sign(z) * s / 2
    nn = (x - cen) / np.linalg.norm(x - cen, axis=1, keepdims=True)
    assert np.abs(n - nn).max() < 2e-5
    # without the sign in the gradient the lower lobe's normals are wrong
    plain, _, _ = oracle.query_scaled(lut, d, scale=s)
    lower = z < 0
    assert np.allclose(out[lower, 1:], -plain[lower, 1:], atol=0, rtol=0)


def test_scaled_radius_properties():
    """R = s r: the normal does not depend on s; a positive function gives
    the same result signed or not."""
    c = workloads.sh_glyph_coeffs(6, 1, rng(81))[0]
    lut = oracle.bake_sh(c, 12)
    d = workloads.uniform_dirs(500, rng(82))
    o1, n1, s1 = oracle.query_scaled(lut, d, scale=1.0)
    o2, n2, _ = oracle.query_scaled(lut, d, scale=2.5)
    o3, n3, s3 = oracle.query_scaled(lut, d, scale=2.5, signed=True)
    base = oracle.query(lut, d)
    np.testing.assert_allclose(o1, base, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(o2, 2.5 * o1, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(n2, n1, atol=1e-14)
    assert (o1[:, 0] > 0).all() and (s1 == 1).all() and (s3 == 1).all()
    np.testing.assert_array_equal(o3, o2)
    np.testing.assert_array_equal(n3, n2)


def test_bisect_budget_definition():
    """The budget is the fewest halvings that bring the march bracket's
    projected width e = 2 rmax px / (depth n_march) to <= eps pixels, capped;
    it grows with the projected size (Sec. 3.1).  Checked against the
    definition in FP64 (the FP32 decision may differ only where e 2^-k is
    within rounding of eps)."""
    r = rng(83)
    cen = np.array([0.1, -0.2, 0.3], np.float32)
    for _ in range(400):
        o = (cen + r.normal(size=3) * r.uniform(0.5, 200)).astype(np.float32)
        rmax, px, eps = float(r.uniform(0.1, 2)), float(r.uniform(50, 4000)), float(r.choice([0.0625, 0.125, 0.5]))
        k = oracle.bisect_budget(o, cen, rmax, px, eps, 20, 16)
        depth = np.linalg.norm(o.astype(np.float64) - cen.astype(np.float64))
        e = 2 * rmax * px / (depth * 20)
        assert 0 <= k <= 16
        if k < 16:
            assert e * 2.0 ** -k <= eps * (1 + 1e-6)
        if k > 0:
            assert e * 2.0 ** -(k - 1) > eps * (1 - 1e-6)
    o = np.array([0, 0, 5], np.float32)
    ks = [oracle.bisect_budget(o, np.zeros(3), 1.0, px, 0.125, 20, 16) for px in (10, 100, 1000, 10000, 1e6)]
    assert ks == sorted(ks) and ks[0] < ks[-1] == 16
    assert oracle.bisect_budget(o, np.zeros(3), 1.0, 0.0, 0.125, 20, 11) == 11


def test_trace_signed_two_spheres_and_budget():
    N, s = 48, 0.5
    lut = z_lut(N)
    rmax = s * oracle.rmax_bound(lut, absval=True)
    assert s <= rmax < 1.01 * s  # max |z| = 1
    r = rng(84)
    P = 400
    o = np.tile(np.array([[1.6, 0.3, 0.1]]), (P, 1))
    tgt = np.stack([np.zeros(P), r.uniform(-0.3, 0.3, P), r.uniform(-0.55, 0.55, P)], axis=1) * s
    dvec = tgt - o
    o32, d32 = o.astype(np.float32), dvec.astype(np.float32)
    t, out, n, sg, ev = oracle.trace_ex(lut, np.zeros(3), rmax, o32, d32, scale=s, signed=True)
    oo, dd = o32.astype(np.float64), d32.astype(np.float64)
    dd /= np.linalg.norm(dd, axis=1, keepdims=True)
    # first hit of the two spheres; grazing rays and hits near the kink are skipped
    best = np.full(P, np.inf)
    clear = np.ones(P, bool)
    for zc in (s / 2, -s / 2):
        oc = oo - np.array([0, 0, zc])
        b = np.einsum("ij,ij->i", oc, dd)
        disc = b * b - (np.einsum("ij,ij->i", oc, oc) - (s / 2) ** 2)
        clear &= np.abs(disc) > 0.05 * (s / 2) ** 2
        th = np.where(disc > 0, -b - np.sqrt(np.maximum(disc, 0)), np.inf)
        best = np.minimum(best, th)
    xh = oo + best[:, None] * dd
    ok = clear & np.isfinite(best) & (np.abs(xh[:, 2]) > 0.05 * s)
    assert ok.sum() > 150
    np.testing.assert_array_equal(np.isfinite(t[clear]), np.isfinite(best[clear]))
    np.testing.assert_allclose(t[ok], best[ok], rtol=1e-6)
    assert np.array_equal(sg[ok], np.sign(xh[ok, 2]).astype(np.int8))
    xo = xh[ok]
    cen = np.zeros_like(xo)
    cen[:, 2] = np.sign(xo[:, 2]) * s / 2
    nn = (xo - cen) / np.linalg.norm(xo - cen, axis=1, keepdims=True)
    assert np.abs(n[ok] - nn).max() < 1e-4
    # every hit spends march + budget + Newton + 1 evaluations
    hit = np.isfinite(t)
    assert (ev[hit] >= 16 + 3 + 2).all() and (ev[hit] <= 20 + 16 + 3 + 1).all()
    # adaptive budget: a small projected size spends fewer bisections, each
    # hit exactly march + k + Newton + 1 with k from the budget rule
    px = 200.0
    k = oracle.bisect_budget(o32[0], np.zeros(3), rmax, px, 0.125, 20, 16)
    assert 0 < k < 16
    ta, _, _, _, eva = oracle.trace_ex(lut, np.zeros(3), rmax, o32, d32, scale=s, signed=True, px=px)
    tk, _, _, _, evk = oracle.trace_ex(lut, np.zeros(3), rmax, o32, d32, scale=s, signed=True, n_bisect=k)
    np.testing.assert_array_equal(ta, tk)
    np.testing.assert_array_equal(eva, evk)
    assert (eva[hit] == ev[hit] - (16 - k)).all()


def test_trace_hits_are_first_roots():
    N = 16
    c = workloads.sh_glyph_coeffs(8, 1, rng(27))[0]
    lut = oracle.bake_sh(c, N)
    rmax = oracle.rmax_bound(lut)
    o, d = workloads.camera_rays(48, 36, eye=(0.3, 0.2, 3.5))
    t, out, n = oracle.trace(lut, np.zeros(3), rmax, o, d)
    hit = np.isfinite(t)
    assert 0.2 < hit.mean() < 0.9
    bad_first = 0
    for k in np.flatnonzero(hit)[::7]:
        F = oracle.trace_F(lut, np.zeros(3), o[k].astype(float), d[k].astype(float), np.array([t[k]]))
        assert abs(F[0]) < 1e-10 * rmax
        # dense scan from the entry of the bounding sphere up to t
        oo = o[k].astype(float)
        dd = d[k].astype(float) / np.linalg.norm(d[k].astype(float))
        bq = oo @ dd
        t0 = max(-bq - math.sqrt(bq * bq - (oo @ oo - rmax * rmax)), 0.0)
        ts = np.linspace(t0, t[k], 4096)[:-2]
        Fs = oracle.trace_F(lut, np.zeros(3), oo, dd, ts)
        bad_first += int((Fs < 0).any())
    assert bad_first <= 1
    # misses: F stays positive along a dense scan of the bounding interval
    for k in np.flatnonzero(~hit)[::50]:
        oo = o[k].astype(float)
        dd = d[k].astype(float) / np.linalg.norm(d[k].astype(float))
        bq = oo @ dd
        disc = bq * bq - (oo @ oo - rmax * rmax)
        if disc < 0:
            continue
        ts = np.linspace(-bq - math.sqrt(disc), -bq + math.sqrt(disc), 2048)
        assert (oracle.trace_F(lut, np.zeros(3), oo, dd, ts) > -1e-3).all()


# ---------------------------------------------------------------------------
# Backward (differentiation form)
# ---------------------------------------------------------------------------
def test_backward_adjoint_identity():
    N = 10
    r = rng(28)
    lut = workloads.random_lut(N, r).astype(np.float64)
    d = workloads.uniform_dirs(3000, r)
    g = r.standard_normal((3000, 4))
    dl = r.standard_normal(lut.shape)
    gl, _ = oracle.backward(lut, d, g, want_dirs=False)
    lhs = np.sum(oracle.query(dl, d) * g)  # forward is linear in the LUT
    rhs = np.sum(dl * gl)
    assert abs(lhs - rhs) < 1e-11 * max(abs(lhs), 1.0) * 10


def test_backward_lut_fd_on_texels():
    N = 8
    r = rng(29)
    lut = workloads.random_lut(N, r).astype(np.float64)
    d = workloads.uniform_dirs(4000, r)
    g = r.standard_normal((4000, 4))
    gl, _ = oracle.backward(lut, d, g, want_dirs=False)
    eps = 1e-3
    for _ in range(64):
        idx = tuple(int(r.integers(s)) for s in lut.shape)
        lp = lut.copy()
        lp[idx] += eps
        lm = lut.copy()
        lm[idx] -= eps
        fd = (np.sum(oracle.query(lp, d) * g) - np.sum(oracle.query(lm, d) * g)) / (2 * eps)
        assert abs(fd - gl[idx]) < 1e-7 * max(1.0, abs(fd))


def test_backward_dirs_fd_and_homogeneity():
    N = 12
    r = rng(30)
    c = workloads.sh_glyph_coeffs(6, 1, r)[0]
    lut = oracle.bake_sh(c, N)
    d = workloads.uniform_dirs(1500, r)
    f, i0, j0, s, t = oracle.locate(d, N)
    keep = (s > 0.02) & (s < 0.98) & (t > 0.02) & (t < 0.98)
    d = d[keep]
    g = r.standard_normal((d.shape[0], 4))
    _, gd = oracle.backward(lut, d, g, want_lut=False)
    dd = d.astype(np.float64)
    # 0-homogeneous outputs: grad_d . d = 0
    scale = np.abs(gd).max()
    assert np.abs(np.einsum("ij,ij->i", gd, dd)).max() < 1e-11 * scale
    h = 1e-7
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        Lp = np.sum(oracle.query_f64(lut, dd + e) * g, axis=1)
        Lm = np.sum(oracle.query_f64(lut, dd - e) * g, axis=1)
        fd = (Lp - Lm) / (2 * h)
        assert np.abs(fd - gd[:, k]).max() < 1e-5 * scale


# ---------------------------------------------------------------------------
# Batched form
# ---------------------------------------------------------------------------
def test_batched_equals_per_object():
    r = rng(31)
    Ns = [4, 9, 16]
    luts = [workloads.random_lut(N, r).astype(np.float64) for N in Ns]
    counts = [100, 1, 250]
    dirs = workloads.uniform_dirs(sum(counts), r)
    off = np.cumsum([0] + [l.size // 4 for l in luts])[:-1]
    qb = np.cumsum([0] + counts)[:-1]
    flat = np.concatenate([l.reshape(-1) for l in luts])
    out = oracle.query_objects(flat, off, Ns, qb, counts, dirs)
    for k in range(3):
        ref = oracle.query(luts[k], dirs[qb[k]:qb[k] + counts[k]])
        assert np.array_equal(out[qb[k]:qb[k] + counts[k]], ref)


# ---------------------------------------------------------------------------
# Bump-field target (radial impostor workload)
# ---------------------------------------------------------------------------
def test_bumps_truth_and_bake_against_independent_evaluation():
    """Values against the generator's independent numpy evaluation; the
    spherical gradient and the baked chart channels against finite
    differences of that evaluation."""
    mu, amp, width = workloads.bump_params(rng(50), 12)
    d = workloads.uniform_dirs(500, rng(51)).astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    tr = oracle.bumps_truth(mu, amp, width, 1.0, d)
    np.testing.assert_allclose(tr[:, 0], workloads.bumps_value(mu, amp, width, 1.0, d), rtol=1e-14)
    tau = np.cross(d, np.array([0.2, -0.4, 0.9]))
    tau /= np.linalg.norm(tau, axis=1, keepdims=True)
    h = 1e-6
    fd = (workloads.bumps_value(mu, amp, width, 1.0, d + h * tau) - workloads.bumps_value(mu, amp, width, 1.0, d - h * tau)) / (2 * h)
    assert np.abs(fd - np.sum(tr[:, 1:] * tau, axis=1)).max() < 1e-6
    assert np.abs(np.sum(tr[:, 1:] * d, axis=1)).max() < 1e-12
    N = 16
    lut = oracle.bake_bumps(mu, amp, width, 1.0, N)
    hh = 1e-4
    r = rng(52)
    for _ in range(30):
        face = int(r.integers(6))
        p, q = int(r.integers(N + 2)), int(r.integers(N + 2))
        u, v = (p - 0.5) / N, (q - 0.5) / N

        def G(uu, vv):
            return workloads.bumps_value(mu, amp, width, 1.0, chart_dir(face, np.array([uu]), np.array([vv])))[0]

        ch = lut[face, q, p]
        assert abs(ch[0] - G(u, v)) < 1e-14
        assert abs(ch[1] - (G(u + hh, v) - G(u - hh, v)) / (2 * hh) / N) < 1e-7
        assert abs(ch[2] - (G(u, v + hh) - G(u, v - hh)) / (2 * hh) / N) < 1e-7
        guv = (G(u + hh, v + hh) - G(u + hh, v - hh) - G(u - hh, v + hh) + G(u - hh, v - hh)) / (4 * hh * hh)
        assert abs(ch[3] - guv / N ** 2) < 1e-6


# ---------------------------------------------------------------------------
# Comparison reconstructions (Sec. 4.2 Table psnr_value, Sec. 4.5 Table
# cost_extended): nearest, bilinear + finite-difference normals, Catmull-Rom
# ---------------------------------------------------------------------------
def value_lut(N, fn):
    """Value-only LUT [6, N+4, N+4] of fn(face, u, v), texel p at u=(p-3/2)/N."""
    p = (np.arange(N + 4) - 1.5) / N
    U, V = np.meshgrid(p, p, indexing="xy")
    return np.stack([fn(f, U, V) for f in range(6)])


def check_chart_grad(out, d, f, pu, pv, tol):
    """out's gradient against chart derivatives (pu, pv): grad . e1 = pu and
    grad . e2 = pv, with e1, e2 from finite differences of the chart map."""
    ff, u, v = face_uv(d.astype(np.float64))
    h = 1e-6
    for k in range(len(d)):
        e1 = (chart_dir(ff[k], u[k] + h, v[k]) - chart_dir(ff[k], u[k] - h, v[k])) / (2 * h)
        e2 = (chart_dir(ff[k], u[k], v[k] + h) - chart_dir(ff[k], u[k], v[k] - h)) / (2 * h)
        assert abs(out[k, 1:] @ e1 - pu[k]) < tol and abs(out[k, 1:] @ e2 - pv[k]) < tol


def test_bilinear_fd_reproduces_bilinear_functions():
    N = 9
    r = rng(60)
    C = r.standard_normal((6, 4))
    vl = value_lut(N, lambda f, U, V: C[f, 0] + C[f, 1] * U + C[f, 2] * V + C[f, 3] * U * V)
    d = workloads.uniform_dirs(400, r)
    out = oracle.baseline_query(vl, d, oracle.BASELINE_BILINEAR_FD)
    f, u, v = face_uv(d.astype(np.float64))
    np.testing.assert_allclose(out[:, 0], C[f, 0] + C[f, 1] * u + C[f, 2] * v + C[f, 3] * u * v, atol=1e-12)
    check_chart_grad(out, d, f, C[f, 1] + C[f, 3] * v, C[f, 2] + C[f, 3] * u, 1e-6)


def test_catmull_rom_reproduces_biquadratics():
    N = 7
    r = rng(61)
    C = r.standard_normal((6, 3, 3))
    def P(f, U, V, du=0, dv=0):
        out = 0.0
        for a in range(3):
            for b in range(3):
                ca = (a if du else 1) * (U ** (a - du) if a >= du else 0)
                cb = (b if dv else 1) * (V ** (b - dv) if b >= dv else 0)
                out = out + C[f, a, b] * ca * cb
        return out
    vl = value_lut(N, lambda f, U, V: P(f, U, V))
    d = workloads.uniform_dirs(400, r)
    out = oracle.baseline_query(vl, d, oracle.BASELINE_BICUBIC)
    f, u, v = face_uv(d.astype(np.float64))
    np.testing.assert_allclose(out[:, 0], [P(ff, uu, vv) for ff, uu, vv in zip(f, u, v)], atol=1e-12)
    check_chart_grad(out, d, f, [P(ff, uu, vv, du=1) for ff, uu, vv in zip(f, u, v)],
                     [P(ff, uu, vv, dv=1) for ff, uu, vv in zip(f, u, v)], 1e-6)


def test_fast_bicubic_is_the_cubic_bspline():
    """The cubic B-spline of the samples reproduces linear and bilinear
    functions exactly, and adds its second moment to a quadratic:
    sum_k k^2 B(x - k) = x^2 + 1/3 in texel units, so U^2 (U = u) comes out
    as U^2 + 1/(3 N^2).  The gradient is the bilinear central difference,
    exact on bilinear functions."""
    N = 9
    r = rng(65)
    C = r.standard_normal((6, 6))
    vl = value_lut(N, lambda f, U, V: C[f, 0] + C[f, 1] * U + C[f, 2] * V + C[f, 3] * U * V)
    d = workloads.uniform_dirs(400, r)
    out = oracle.baseline_query(vl, d, oracle.BASELINE_FAST_BICUBIC_FD)
    f, u, v = face_uv(d.astype(np.float64))
    np.testing.assert_allclose(out[:, 0], C[f, 0] + C[f, 1] * u + C[f, 2] * v + C[f, 3] * u * v, atol=1e-12)
    check_chart_grad(out, d, f, C[f, 1] + C[f, 3] * v, C[f, 2] + C[f, 3] * u, 1e-6)
    vq = value_lut(N, lambda f, U, V: C[f, 0] + C[f, 4] * U * U + C[f, 5] * V * V)
    out = oracle.baseline_query(vq, d, oracle.BASELINE_FAST_BICUBIC_FD)
    want = C[f, 0] + C[f, 4] * (u * u + 1 / (3 * N * N)) + C[f, 5] * (v * v + 1 / (3 * N * N))
    np.testing.assert_allclose(out[:, 0], want, atol=1e-12)


def test_nearest_returns_texel_values():
    N = 6
    r = rng(62)
    vl = r.standard_normal((6, N + 4, N + 4))
    d = workloads.uniform_dirs(300, r)
    out = oracle.baseline_query(vl, d, oracle.BASELINE_NEAREST)
    f, u, v = face_uv(d.astype(np.float64))
    p = np.floor(u * N + 1.5 + 0.5).astype(int)
    q = np.floor(v * N + 1.5 + 0.5).astype(int)
    np.testing.assert_array_equal(out[:, 0], vl[f, q, p])
    assert np.all(out[:, 1:] == 0)


def test_value_psnr_ordering_matches_table_psnr_value():
    """Table psnr_value: Hermite > Catmull-Rom bicubic > bilinear at every N,
    with gains per doubling of roughly +12 dB (bilinear), +22 dB (bicubic),
    +30 dB (Hermite) between N = 8, 16, 32."""
    c = workloads.sh_glyph_coeffs(8, 1, rng(63))[0]
    d = workloads.uniform_dirs(30000, rng(64))
    truth = oracle.sh_truth(c, d.astype(np.float64))[:, 0]
    peak = truth.max() - truth.min()
    psnr = {}
    for N in (8, 16, 32):
        vl = oracle.sh_truth(c, oracle.margin_dirs(N).reshape(-1, 3))[:, 0].reshape(6, N + 4, N + 4)
        for name, m in (("bilinear", oracle.BASELINE_BILINEAR_FD), ("bicubic", oracle.BASELINE_BICUBIC)):
            e = oracle.baseline_query(vl, d, m)[:, 0] - truth
            psnr[(name, N)] = 20 * math.log10(peak / np.sqrt(np.mean(e ** 2)))
        e = oracle.query(oracle.bake_sh(c, N), d)[:, 0] - truth
        psnr[("hermite", N)] = 20 * math.log10(peak / np.sqrt(np.mean(e ** 2)))
    paper = {int(row[0]): row[1:] for row in load_golden("psnr_value_table.txt")}
    for N in (8, 16, 32):
        assert psnr[("hermite", N)] > psnr[("bicubic", N)] > psnr[("bilinear", N)], (N, psnr)
        assert paper[N][2] > paper[N][1] > paper[N][0]
    gains = {m: psnr[(m, 32)] - psnr[(m, 16)] for m in ("bilinear", "bicubic", "hermite")}
    assert 9 < gains["bilinear"] < 15, gains      # second order: ~12 dB
    assert 15 < gains["bicubic"] < 27, gains      # paper: 21.5 dB
    assert gains["hermite"] > gains["bicubic"]


# ---------------------------------------------------------------------------
# Mip chain (Sec. 4.7, Table lod)
# ---------------------------------------------------------------------------
def test_mip_constant_and_box_filter():
    N = 8
    lut = np.zeros((6, N + 2, N + 2, 4))
    lut[..., 0] = 0.9
    for naive in (False, True):
        m = oracle.mip_level(lut, naive=naive)
        assert np.abs(m[..., 0] - 0.9).max() < 1e-13 and np.abs(m[..., 1:]).max() < 1e-13
    lut = workloads.random_lut(N, rng(70)).astype(np.float64)
    box = 0.25 * (lut[:, 1:N + 1:2, 1:N + 1:2] + lut[:, 1:N + 1:2, 2:N + 2:2] + lut[:, 2:N + 2:2, 1:N + 1:2] + lut[:, 2:N + 2:2, 2:N + 2:2])
    c = oracle.mip_level(lut)
    n = oracle.mip_level(lut, naive=True)
    # interior coarse values are the box filter of the fine values (the map
    # reproduces the stored value at every fine texel centre)
    np.testing.assert_allclose(c[:, 1:-1, 1:-1, 0], box[..., 0], atol=1e-13)
    np.testing.assert_allclose(n[:, 1:-1, 1:-1], box, atol=1e-13)
    # gutters are shared by both constructions
    np.testing.assert_array_equal(c[:, 0], n[:, 0])


def test_mip_table_lod_trend():
    """Table lod: naive box filtering of the derivative channels is several
    times worse at the first coarse level (5.5x in the paper), the gap
    closing at coarser levels (2.9x, 1.3x)."""
    c = workloads.sh_glyph_coeffs(8, 1, rng(71))[0]
    d = workloads.uniform_dirs(20000, rng(72))
    w = d.astype(np.float64)
    w /= np.linalg.norm(w, axis=1, keepdims=True)

    def normals(out):
        n = out[:, :1] * w - out[:, 1:]
        return n / np.linalg.norm(n, axis=1, keepdims=True)

    tn = normals(oracle.sh_truth(c, w))

    def err(lut):
        return np.degrees(np.arccos(np.clip(np.sum(normals(oracle.query(lut, d)) * tn, axis=1), -1, 1))).mean()

    cons = naive = oracle.bake_sh(c, 32)
    ratios = []
    for _ in range(3):
        cons, naive = oracle.mip_level(cons), oracle.mip_level(naive, naive=True)
        ratios.append(err(naive) / err(cons))
    assert ratios[0] > 3.0, ratios
    assert ratios[0] > ratios[1] > ratios[2] > 1.0, ratios


# ---------------------------------------------------------------------------
# Radial depth of a mesh (Sec. 4.9): R(w) = max{t >= 0 : c + t w on the mesh}
# ---------------------------------------------------------------------------
def box_mesh(lo, hi):
    """Axis-aligned box as 12 triangles."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    V = np.array([[hi[0] if i & 1 else lo[0], hi[1] if i & 2 else lo[1], hi[2] if i & 4 else lo[2]] for i in range(8)])
    quads = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    F = [(a, b, c) for a, b, c, d in quads] + [(a, c, d) for a, b, c, d in quads]
    return V, np.array(F, np.int32)


def test_mesh_depth_cube_and_octahedron_closed_forms():
    a, c = 0.7, np.array([0.3, -1.2, 2.0])
    V, F = box_mesh(c - a, c + a)
    d = np.concatenate([workloads.uniform_dirs(3000, rng(90)), oracle.margin_dirs(8).reshape(-1, 3)]).astype(np.float32)
    w = d.astype(np.float64) / np.linalg.norm(d.astype(np.float64), axis=1, keepdims=True)
    R = oracle.mesh_radial_depth(V, F, c, d)
    np.testing.assert_allclose(R, a / np.abs(w).max(axis=1), rtol=1e-12)
    Vo = np.array([[a, 0, 0], [-a, 0, 0], [0, a, 0], [0, -a, 0], [0, 0, a], [0, 0, -a]])
    Fo = np.array([(i, j, k) for i in (0, 1) for j in (2, 3) for k in (4, 5)], np.int32)
    R = oracle.mesh_radial_depth(Vo, Fo, np.zeros(3), d)
    np.testing.assert_allclose(R, a / np.abs(w).sum(axis=1), rtol=1e-12)


def test_mesh_depth_takes_the_farthest_hit():
    """Two nested shells: every ray crosses both, the depth is the outer one;
    a box that does not contain the centre gives the exit distance of the
    slab test where the ray meets it and 0 elsewhere; triangles with an
    index out of range are ignored."""
    Vi, Fi = box_mesh([-0.5] * 3, [0.5] * 3)
    Vo, Fo = box_mesh([-1.0] * 3, [1.0] * 3)
    V = np.concatenate([Vi, Vo])
    F = np.concatenate([Fi, Fo + 8]).astype(np.int32)
    d = workloads.uniform_dirs(2000, rng(91))
    w = d.astype(np.float64) / np.linalg.norm(d.astype(np.float64), axis=1, keepdims=True)
    np.testing.assert_allclose(oracle.mesh_radial_depth(V, F, np.zeros(3), d), 1.0 / np.abs(w).max(axis=1), rtol=1e-12)
    lo, hi = np.array([1.0, -0.6, -0.4]), np.array([2.5, 0.7, 0.5])
    Vb, Fb = box_mesh(lo, hi)
    R = oracle.mesh_radial_depth(Vb, Fb, np.zeros(3), d)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1, t2 = lo[None] / w, hi[None] / w
    tn = np.nanmax(np.minimum(t1, t2), axis=1)
    tf = np.nanmin(np.maximum(t1, t2), axis=1)
    hit = (tn <= tf) & (tf >= 0)
    assert 0.05 < hit.mean() < 0.5
    np.testing.assert_allclose(R[hit], tf[hit], rtol=1e-12)
    assert (R[~hit] == 0).all()
    Fbad = np.concatenate([Fb, [[0, 1, 99], [-1, 2, 3]]]).astype(np.int32)
    np.testing.assert_array_equal(oracle.mesh_radial_depth(Vb, Fbad, np.zeros(3), d), R)


def test_asteroid_mesh_depth_tracks_the_radius():
    """The synthetic asteroid mesh is star-shaped about the origin: along a
    vertex direction the depth is that vertex's radius, and elsewhere it
    stays within the surface's radius range (flat facets cut inside)."""
    prm = workloads.asteroid_params(rng(92))
    V, F = workloads.asteroid_mesh(prm, level=3)
    R = oracle.mesh_radial_depth(V, F, np.zeros(3), V[::7])
    np.testing.assert_allclose(R, np.linalg.norm(V[::7].astype(np.float64), axis=1), rtol=1e-6)
    d = workloads.uniform_dirs(500, rng(93))
    R = oracle.mesh_radial_depth(V, F, np.zeros(3), d)
    r, _ = workloads.asteroid_radius(prm, d)
    assert (R > 0.7).all() and np.abs(R - r).max() < 0.1


def test_fd_baked_hermite_is_catmull_rom():
    """Cubic Hermite interpolation whose tangents are the central
    differences (p[i+1] - p[i-1]) / 2 is the Catmull-Rom spline, and the
    tensor product carries the mixed channel along; so a map baked in the
    general (finite-difference) mode reproduces the 16-tap Catmull-Rom
    reconstruction of the same samples, value and gradient, everywhere on
    the sphere (gutters included)."""
    N = 12
    r = rng(94)
    samples = 1.0 + 0.2 * r.standard_normal((6, N + 4, N + 4))
    lut = oracle.bake_fd(samples, N)
    d = workloads.uniform_dirs(5000, r)
    h = oracle.query(lut, d)
    cr = oracle.baseline_query(samples, d, oracle.BASELINE_BICUBIC)
    np.testing.assert_allclose(h[:, 0], cr[:, 0], rtol=0, atol=1e-13)
    np.testing.assert_allclose(h[:, 1:], cr[:, 1:], rtol=0, atol=1e-11)


def test_abs_bound_of_a_signed_function():
    """r = z - 0.3 spans about [-1.3, 0.7]: the bound of |r| covers the
    negative lobe, the plain bound only the positive one; both hold over a
    dense set of queries and are tight to the Bezier hull."""
    c = np.zeros(4)
    c[0] = -0.3 * math.sqrt(4 * math.pi)
    c[2] = math.sqrt(4 * math.pi / 3)
    lut = oracle.bake_sh(c, 16)
    r = oracle.query(lut, workloads.uniform_dirs(20000, rng(95)))[:, 0]
    plain, absb = oracle.rmax_bound(lut), oracle.rmax_bound(lut, absval=True)
    assert plain >= r.max() and absb >= np.abs(r).max()
    assert 0.69 < plain < 0.72 and 1.29 < absb < 1.32
    assert oracle.rmax_bound(-lut, absval=True) == absb
