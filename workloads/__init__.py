"""Seeded synthetic inputs for the Spherical Hermite Maps workloads.

This module holds no arithmetic of the method itself (no cubemap mapping, no
bake, no Hermite reconstruction, no gradient transport): it draws random
numbers and evaluates the *target* functions that a user would hand to the
method (SH coefficient vectors, Gaussian bumps, value-noise heightfields),
plus camera rays.  Both the FP64 oracle and the GPU library consume what it
produces; neither imports the other.

Every generator takes a ``numpy.random.Generator`` (PCG64).  The canonical
workloads use seed 20063 + k for workload k (k = 1..5).

Workloads (all synthetic; the paper's own glyph seed, dMRI data, asteroid
mesh and planet generator are not available, these stand in for them):
  1  one SH glyph, L=4, face N=10, 65,536 uniform directions
  2  32,768 SH glyphs, L=8, N=32, 256 uniform directions per glyph
  3  one radial impostor, 64 Gaussian bumps on radius 1, N=256,
     1920x1080 primary rays
  4  fBm heightfield target 1 + 0.2 fBm(w), 2^22 directions, N=512
  5  4,096 uneven objects, N in {8..256}, L in {2..16}, lognormal counts
"""
import functools
import math

import numpy as np

SEED_BASE = 20063


def rng_for(workload):
    return np.random.default_rng(SEED_BASE + int(workload))


# --------------------------------------------------------------------------
# directions
# --------------------------------------------------------------------------
def uniform_dirs(n, rng):
    """Uniform on the sphere: normalised N(0, I3), drawn in FP64 and rounded
    once to FP32 (the rounded vectors are the inputs; they are not
    renormalised)."""
    g = rng.standard_normal((n, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return g.astype(np.float32)


# --------------------------------------------------------------------------
# SH glyph coefficients
# --------------------------------------------------------------------------
def sh_degree_of_index(L):
    return np.concatenate([np.full(2 * l + 1, l) for l in range(L + 1)])


def fibonacci_sphere(n=4096):
    """n points of the golden-angle (Fibonacci) spiral on the unit sphere:
    z_i = 1 - (2 i + 1)/n, azimuth i pi (3 - sqrt 5).  FP64 [n, 3]."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def real_sh(L, dirs):
    """Orthonormal real spherical harmonics Y_k(w), k = l^2 + l + m, without
    the Condon-Shortley phase (Y_1,1 ~ +x, Y_1,-1 ~ +y), at unit directions
    dirs [n, 3] (FP64); from scipy's complex harmonics (which carry the
    phase (-1)^m):  Y_l,+m = sqrt2 (-1)^m Re Y_l^m,  Y_l,-m = sqrt2 (-1)^m
    Im Y_l^m,  Y_l,0 = Y_l^0.  Returns [n, (L+1)^2] FP64.  This is the
    convention the target functions are written in (the generator needs it
    for the normalisation of the glyphs, nothing else)."""
    from scipy.special import sph_harm_y

    d = np.asarray(dirs, np.float64).reshape(-1, 3)
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))  # polar
    phi = np.arctan2(d[:, 1], d[:, 0])               # azimuth
    Y = np.empty((d.shape[0], (L + 1) ** 2))
    for l in range(L + 1):
        Y[:, l * l + l] = sph_harm_y(l, 0, theta, phi).real
        for m in range(1, l + 1):
            z = sph_harm_y(l, m, theta, phi) * ((-1.0) ** m) * math.sqrt(2.0)
            Y[:, l * l + l + m] = z.real
            Y[:, l * l + l - m] = z.imag
    return Y


@functools.lru_cache(maxsize=None)
def _fibonacci_basis(L):
    """real_sh(L) at the 4,096-point Fibonacci sphere (read-only, cached:
    the uneven batch draws 4,096 glyphs one at a time)."""
    Y = real_sh(L, fibonacci_sphere(4096))
    Y.setflags(write=False)
    return Y


def sh_glyph_coeffs(L, n_obj, rng):
    """Coefficients c_lm = z / (1 + l)^2, z ~ N(0, 1), then the affine map
    R = 1 + 0.3 SH / max|SH| folded in, max|SH| taken over the 4,096-point
    Fibonacci sphere in FP64; R then spans [0.7, 1.3] on those points (the
    extremes of the sphere may lie slightly beyond).  Y_00 = 1 / (2 sqrt(pi)),
    so the constant 1 is c_00 += 2 sqrt(pi).
    Returns FP64 [n_obj, (L+1)^2]; index k = l^2 + l + m."""
    K = (L + 1) ** 2
    lk = sh_degree_of_index(L)
    c = rng.standard_normal((n_obj, K)) / (1.0 + lk) ** 2
    Y = _fibonacci_basis(L)
    M = np.empty(n_obj)
    for o0 in range(0, n_obj, 4096):  # [4096 x K] x [K x chunk]
        M[o0:o0 + 4096] = np.abs(Y @ c[o0:o0 + 4096].T).max(axis=0)
    c = 0.3 * c / M[:, None]
    c[:, 0] += 2.0 * math.sqrt(math.pi)
    return c


# --------------------------------------------------------------------------
# Gaussian bumps (workload 3)
# --------------------------------------------------------------------------
def bump_params(rng, K=64):
    """Centres uniform on the sphere, amplitudes U[0.02, 0.15], widths
    U[0.05, 0.4] rad; the bump is a exp((w . mu - 1) / width^2) (von
    Mises-Fisher form, ~ exp(-theta^2 / (2 width^2)) near its centre)."""
    mu = rng.standard_normal((K, 3))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    amp = rng.uniform(0.02, 0.15, K)
    width = rng.uniform(0.05, 0.4, K)
    return mu, amp, width


def bumps_value(mu, amp, width, base, dirs):
    """R(w) = base + sum_k amp_k exp((w . mu_k - 1) / width_k^2), w = d/|d|."""
    d = np.asarray(dirs, np.float64).reshape(-1, 3)
    w = d / np.linalg.norm(d, axis=1, keepdims=True)
    out = np.full(w.shape[0], float(base))
    for k in range(len(amp)):
        out += amp[k] * np.exp((w @ mu[k] - 1.0) / (width[k] ** 2))
    return out


def camera_rays(width=1920, height=1080, eye=(0.0, 0.0, 3.5), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), vfov_deg=40.0):
    """Pinhole camera, one ray per pixel centre (row-major, top row first).
    Returns origins [P, 3] and unit directions [P, 3], FP32."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    upv = np.cross(right, fwd)
    th = math.tan(math.radians(vfov_deg) / 2.0)
    aspect = width / height
    px = (np.arange(width) + 0.5) / width * 2.0 - 1.0
    py = 1.0 - (np.arange(height) + 0.5) / height * 2.0
    X, Y = np.meshgrid(px * th * aspect, py * th)
    d = fwd[None, None, :] + X[..., None] * right[None, None, :] + Y[..., None] * upv[None, None, :]
    d = d.reshape(-1, 3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.broadcast_to(eye, d.shape)
    return np.ascontiguousarray(o, np.float32), np.ascontiguousarray(d, np.float32)


# --------------------------------------------------------------------------
# fBm value-noise heightfield (workload 4)
# --------------------------------------------------------------------------
def _hash3(ix, iy, iz, seed):
    """32-bit integer hash of a lattice point -> U[-1, 1] (murmur3 finaliser)."""
    h = (ix.astype(np.uint32) * np.uint32(0x8DA6B343)) ^ (iy.astype(np.uint32) * np.uint32(0xD8163841)) \
        ^ (iz.astype(np.uint32) * np.uint32(0xCB1AB31F)) ^ np.uint32(seed)
    h ^= h >> np.uint32(16)
    h *= np.uint32(0x85EBCA6B)
    h ^= h >> np.uint32(13)
    h *= np.uint32(0xC2B2AE35)
    h ^= h >> np.uint32(16)
    return h.astype(np.float64) / 4294967295.0 * 2.0 - 1.0


def _fade(x):
    return x * x * x * (x * (x * 6.0 - 15.0) + 10.0)


def _dfade(x):
    return 30.0 * x * x * (x * (x - 2.0) + 1.0)


def value_noise(p, seed):
    """Trilinear value noise with quintic fade; returns value [n] and the
    ambient gradient [n, 3]."""
    with np.errstate(over="ignore"):
        fl = np.floor(p)
        i = fl.astype(np.int64)
        f = p - fl
        w = _fade(f)
        dw = _dfade(f)
        val = np.zeros(p.shape[0])
        grad = np.zeros_like(p)
        for cx in (0, 1):
            for cy in (0, 1):
                for cz in (0, 1):
                    h = _hash3(i[:, 0] + cx, i[:, 1] + cy, i[:, 2] + cz, seed)
                    wx = w[:, 0] if cx else 1.0 - w[:, 0]
                    wy = w[:, 1] if cy else 1.0 - w[:, 1]
                    wz = w[:, 2] if cz else 1.0 - w[:, 2]
                    sx = 1.0 if cx else -1.0
                    sy = 1.0 if cy else -1.0
                    sz = 1.0 if cz else -1.0
                    val += h * wx * wy * wz
                    grad[:, 0] += h * sx * dw[:, 0] * wy * wz
                    grad[:, 1] += h * wx * sy * dw[:, 1] * wz
                    grad[:, 2] += h * wx * wy * sz * dw[:, 2]
    return val, grad


def fbm_target(dirs, seed, octaves=6, lacunarity=2.0, gain=0.5, f0=2.0, amp=0.2):
    """R*(w) = 1 + amp * fBm(w), fBm = sum_o gain^o noise(lacunarity^o f0 w)
    / sum_o gain^o.  Returns R* [n] and its spherical gradient [n, 3] (the
    tangential part of the ambient gradient at the unit direction)."""
    d = np.asarray(dirs, np.float64).reshape(-1, 3)
    w = d / np.linalg.norm(d, axis=1, keepdims=True)
    val = np.zeros(w.shape[0])
    grad = np.zeros_like(w)
    norm = sum(gain ** o for o in range(octaves))
    for o in range(octaves):
        freq = f0 * lacunarity ** o
        v, g = value_noise(w * freq, seed + 101 * o)
        val += gain ** o * v
        grad += gain ** o * freq * g
    val = 1.0 + amp * val / norm
    grad = amp * grad / norm
    grad -= np.sum(grad * w, axis=1, keepdims=True) * w
    return val, grad


def _mul32(h, c):
    """(h * c) mod 2^32 for 0 <= h < 2^32 held in int64, without overflow."""
    lo = c & 0xFFFF
    hi = c >> 16
    return (h * lo + (((h * hi) & 0xFFFF) << 16)) & 0xFFFFFFFF


def fbm_target_torch(dirs, seed, octaves=6, lacunarity=2.0, gain=0.5, f0=2.0, amp=0.2):
    """The same target as fbm_target, evaluated with torch (any device, FP64);
    returns (R* [n], spherical gradient [n, 3])."""
    import torch

    d = dirs.to(torch.float64)
    w = d / torch.linalg.norm(d, dim=1, keepdim=True)
    val = torch.zeros(w.shape[0], dtype=torch.float64, device=w.device)
    grad = torch.zeros_like(w)
    norm = sum(gain ** o for o in range(octaves))
    M = 0xFFFFFFFF
    for o in range(octaves):
        freq = f0 * lacunarity ** o
        p = w * freq
        fl = torch.floor(p)
        i = fl.to(torch.int64)
        f = p - fl
        wt = _fade(f)
        dwt = _dfade(f)
        s = (seed + 101 * o) & M
        for cx in (0, 1):
            for cy in (0, 1):
                for cz in (0, 1):
                    h = _mul32((i[:, 0] + cx) & M, 0x8DA6B343) ^ _mul32((i[:, 1] + cy) & M, 0xD8163841) \
                        ^ _mul32((i[:, 2] + cz) & M, 0xCB1AB31F) ^ s
                    h = h ^ (h >> 16)
                    h = _mul32(h, 0x85EBCA6B)
                    h = h ^ (h >> 13)
                    h = _mul32(h, 0xC2B2AE35)
                    h = h ^ (h >> 16)
                    hv = h.to(torch.float64) / 4294967295.0 * 2.0 - 1.0
                    wx = wt[:, 0] if cx else 1.0 - wt[:, 0]
                    wy = wt[:, 1] if cy else 1.0 - wt[:, 1]
                    wz = wt[:, 2] if cz else 1.0 - wt[:, 2]
                    sx = 1.0 if cx else -1.0
                    sy = 1.0 if cy else -1.0
                    sz = 1.0 if cz else -1.0
                    v = gain ** o
                    val += v * hv * wx * wy * wz
                    grad[:, 0] += v * freq * hv * sx * dwt[:, 0] * wy * wz
                    grad[:, 1] += v * freq * hv * wx * sy * dwt[:, 1] * wz
                    grad[:, 2] += v * freq * hv * wx * wy * sz * dwt[:, 2]
    val = 1.0 + amp * val / norm
    grad = amp * grad / norm
    grad = grad - torch.sum(grad * w, dim=1, keepdim=True) * w
    return val, grad


# --------------------------------------------------------------------------
# uneven batch (workload 5)
# --------------------------------------------------------------------------
BATCH_NS = (8, 16, 32, 64, 128, 256)
BATCH_NP = (0.3, 0.25, 0.2, 0.15, 0.07, 0.03)


def _rand_unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def asteroid_params(rng):
    """Feature parameters of the synthetic asteroid that stands in for the
    paper's mesh impostor model: 69 craters (6 large, 18 medium, 45 small:
    angular radius, depth), 8 ridges along great circles (plane normal,
    height, half-width), 30 boulders (centre, height, width) and a seed for
    5-octave fBm."""
    craters = [], [], []
    for n, (r0, r1), (d0, d1) in zip((6, 18, 45), ((0.35, 0.55), (0.15, 0.3), (0.05, 0.12)),
                                     ((0.06, 0.10), (0.03, 0.06), (0.01, 0.03))):
        craters[0].append(_rand_unit(rng, n))
        craters[1].append(rng.uniform(r0, r1, n))
        craters[2].append(rng.uniform(d0, d1, n))
    return {"craters": tuple(np.concatenate(c) for c in craters),
            "ridges": (_rand_unit(rng, 8), rng.uniform(0.02, 0.05, 8), rng.uniform(0.04, 0.1, 8)),
            "boulders": (_rand_unit(rng, 30), rng.uniform(0.01, 0.03, 30), rng.uniform(0.02, 0.05, 30)),
            "noise_seed": int(rng.integers(1 << 30))}


def asteroid_radius(prm, dirs):
    """Radius R(w) of the asteroid and its spherical gradient [n, 3]:
    1 + craters (bowl -D e^{-2x} with a rim 0.3 D e^{-(x-1)^2/0.18},
    x = (1 - w.mu)/rho^2) + ridges (h e^{-(w.n/b)^2}) + boulders
    (h e^{(w.c - 1)/s^2}) + 0.05 fBm (5 octaves); R stays in about
    [0.8, 1.15]."""
    d = np.asarray(dirs, np.float64).reshape(-1, 3)
    w = d / np.linalg.norm(d, axis=1, keepdims=True)
    val = np.ones(w.shape[0])
    grad = np.zeros_like(w)
    mu, rho, depth = prm["craters"]
    for k in range(mu.shape[0]):
        x = (1.0 - w @ mu[k]) / rho[k] ** 2
        bowl = np.exp(-2.0 * x)
        rim = np.exp(-(x - 1.0) ** 2 / 0.18)
        val += -depth[k] * bowl + 0.3 * depth[k] * rim
        dfx = 2.0 * depth[k] * bowl - 0.3 * depth[k] * rim * 2.0 * (x - 1.0) / 0.18
        grad += dfx[:, None] * (-mu[k] / rho[k] ** 2)[None, :]
    nrm, hgt, hw = prm["ridges"]
    for k in range(nrm.shape[0]):
        y = w @ nrm[k]
        e = np.exp(-(y / hw[k]) ** 2)
        val += hgt[k] * e
        grad += (hgt[k] * e * (-2.0 * y / hw[k] ** 2))[:, None] * nrm[k][None, :]
    c, h, wd = prm["boulders"]
    for k in range(c.shape[0]):
        e = np.exp((w @ c[k] - 1.0) / wd[k] ** 2)
        val += h[k] * e
        grad += (h[k] * e / wd[k] ** 2)[:, None] * c[k][None, :]
    grad -= np.sum(grad * w, axis=1, keepdims=True) * w
    fv, fg = fbm_target(w, prm["noise_seed"], octaves=5, amp=0.05)
    return val + fv - 1.0, grad + fg


def icosphere(level):
    """Unit icosphere: the icosahedron with every triangle split into four
    `level` times, new vertices pushed to the sphere.  Vertices [V, 3]
    (FP64), outward-oriented triangles [T, 3] (int64); T = 20 * 4^level."""
    p = (1 + 5 ** 0.5) / 2
    v0 = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
          (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
             (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
             (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    V = [np.array(x, float) / np.linalg.norm(x) for x in v0]
    F = faces
    for _ in range(level):
        mids = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in mids:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                mids[key] = len(V) - 1
            return mids[key]

        nf = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nf
    return np.array(V), np.array(F, np.int64)


def asteroid_mesh(prm, level=6):
    """Star-shaped triangle mesh of the asteroid: icosphere vertices moved to
    radius R(w).  Vertices [V, 3] FP32, triangles [T, 3] int32 (81,920 at
    level 6), centred on the origin."""
    V, F = icosphere(level)
    r, _ = asteroid_radius(prm, V)
    return np.ascontiguousarray(V * r[:, None], np.float32), np.ascontiguousarray(F, np.int32)


def uneven_batch(rng, n_obj=4096, mu=9.0, sigma=1.5, qmin=64, qmax=1 << 20, Lmin=2, Lmax=16):
    """Per object: face size N, SH order L, query count Q (lognormal,
    clipped).  Returns dict of int arrays."""
    Ns = rng.choice(np.array(BATCH_NS), size=n_obj, p=np.array(BATCH_NP))
    Ls = rng.integers(Lmin, Lmax + 1, size=n_obj)
    Q = np.clip(np.rint(rng.lognormal(mu, sigma, size=n_obj)), qmin, qmax).astype(np.int64)
    return {"N": Ns.astype(np.int32), "L": Ls.astype(np.int32), "Q": Q}


# --------------------------------------------------------------------------
# arbitrary LUT contents (the query is defined for any LUT)
# --------------------------------------------------------------------------
def random_lut(N, rng, n_obj=None, base=1.0, spread=0.2):
    """Random texel data in LUT layout [..., 6, N+2, N+2, 4]: values in
    base +- spread, scaled derivative channels of a comparable scale."""
    shape = (6, N + 2, N + 2, 4) if n_obj is None else (n_obj, 6, N + 2, N + 2, 4)
    x = rng.uniform(-1.0, 1.0, shape)
    x[..., 0] = base + spread * x[..., 0]
    x[..., 1] *= 0.5 * spread
    x[..., 2] *= 0.5 * spread
    x[..., 3] *= 0.25 * spread
    return x.astype(np.float32)
