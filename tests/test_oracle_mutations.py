"""Mutation sweep of the oracle pins (CPU only): each case plants one
plausible mistake in a copy of the oracle source (a flipped sign, a dropped
term, a wrong index, offset or scale), builds it, and runs the pins of
tests/test_oracle_pins.py against it in a child process.  Every mutant must
make at least one pin fail; a mutant the pins accept would mean that part of
the oracle is unpinned."""
import concurrent.futures as cf
import os
import subprocess
import sys

import oracle
from conftest import ROOT

PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")

# (name, exact text in shm_oracle.c (must occur once), replacement)
MUTANTS = [
    ("face table sign", "FS[6][3] = {{0, 0, -1},", "FS[6][3] = {{0, 0, 1},"),
    # (the sign test of the major axis cannot see -0: a zero major axis means a
    # zero direction, which is invalid before any face is chosen)
    ("face tie-break order", "if (ax >= ay && ax >= az) return x >= 0.0 ? 0 : 1;",
     "if (ax > ay && ax >= az) return x >= 0.0 ? 0 : 1;"),
    ("face tie-break order Y/Z", "if (ay >= az) return y >= 0.0 ? 2 : 3;", "if (ay > az) return y >= 0.0 ? 2 : 3;"),
    ("texel centre offset", "double fu = (L->a + 1.0) * 0.5 * (double)N + 0.5;\n",
     "double fu = (L->a + 1.0) * 0.5 * (double)N + 0.25;\n"),
    ("Hermite basis term", "Hb[2] = hadd(hsub(s3, hscale(s2, 2.0)), s);", "Hb[2] = hsub(s3, hscale(s2, 2.0));"),
    ("Hermite derivative", "Hd[1] = hadd(hscale(s2, -6.0), hscale(s, 6.0));",
     "Hd[1] = hadd(hscale(s2, -6.0), hscale(s, 5.0));"),
    ("dropped cross term", "            acc = hadd(acc, hscale(hmul(Hdi, Hdj), c[3]));\n", "\n"),
    ("swapped channels", "acc = hadd(acc, hscale(hmul(Hdi, Hj), c[1]));", "acc = hadd(acc, hscale(hmul(Hdi, Hj), c[2]));"),
    ("derivative N scale", "*ru = hscale(accu, (double)N);", "*ru = hscale(accu, (double)(N + 1));"),
    ("tangent uses T for S", "e1[k] = hmul(hsub(hc(2.0 * FS[face][k]), hmul(w[k], wS)), irho);",
     "e1[k] = hmul(hsub(hc(2.0 * FT[face][k]), hmul(w[k], wS)), irho);"),
    ("metric determinant sign", "hd det = hsub(hmul(g11, g22), hmul(g12, g12));",
     "hd det = hadd(hmul(g11, g22), hmul(g12, g12));"),
    ("Cramer sign", "hd alpha = hmul(hsub(hmul(g22, ru), hmul(g12, rv)), idet);",
     "hd alpha = hmul(hadd(hmul(g22, ru), hmul(g12, rv)), idet);"),
    ("normal sign", "m[k] = R * w[k] - g[k];", "m[k] = R * w[k] + g[k];"),
    ("SH phase", "Y[l * l + l - m] = hscale(hmul(Q, B[m]), sqrt(2.0) * K);",
     "Y[l * l + l - m] = hscale(hmul(Q, B[m]), -sqrt(2.0) * K);"),
    ("SH normalisation", "double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * ratio);",
     "double K = sqrt((2.0 * l + 1.0) / (4.5 * M_PI) * ratio);"),
    ("bake derivative scaling", "out4[1] = G.a * h;", "out4[1] = G.a * h * h;"),
    ("bake texel centres (gutter rule)", "double u = ((double)p - 0.5) / (double)N, v = ((double)q - 0.5) / (double)N;",
     "double u = ((double)p - 0.4) / (double)N, v = ((double)q - 0.5) / (double)N;"),
    ("backward scale", "double w = g[4 * q] * r.v;", "double w = 2.0 * g[4 * q] * r.v;"),
    ("direction tangent length", "dd[axis] = 1.0;", "dd[axis] = 2.0;"),
    ("Bezier control point", "b[1] = h[0] + h[1] / 3.0;", "b[1] = h[0] + h[1] / 2.0;"),
    ("march threshold", "if (E.ok && E.F < 0.0) { hit = 1;", "if (E.ok && E.F < -1e-3) { hit = 1;"),
    ("bisection side", "if (E.F < 0.0) hi = mid; else lo = mid;", "if (E.F < 0.0) lo = mid; else hi = mid;"),
    ("Newton sign", "double tn = t - E.F / E.dF;", "double tn = t + E.F / E.dF;"),
    ("budget halving", "while (k < n_bisect && e > eps_px) { e *= 0.5f; ++k; }",
     "while (k < n_bisect && e > eps_px) { e *= 0.25f; ++k; }"),
    ("signed gradient", "double k = signed_ ? s * sg : s;", "double k = s;"),
    ("signed absolute value", "return signed_ ? s * fabs(r) : s * r;", "return s * r;"),
    ("FD bake derivative", "o[1] = 0.5 * (SM(pp + 1, qq) - SM(pp - 1, qq));", "o[1] = 0.25 * (SM(pp + 1, qq) - SM(pp - 1, qq));"),
    ("Catmull-Rom weight", "w[3] = 0.5 * (t3 - t2);", "w[3] = 0.5 * (t3 + t2);"),
    ("B-spline weight", "w[1] = (3 * t3 - 6 * t2 + 4) / 6.0;", "w[1] = (3 * t3 - 6 * t2 + 4) / 5.0;"),
    ("B-spline tap offset", "R += ws[i] * wt[j] * vl_at(vlut, N, f, i0 - 1 + i, j0 - 1 + j);",
     "R += ws[i] * wt[j] * vl_at(vlut, N, f, i0 + i, j0 - 1 + j);"),
    ("mip sub-sample offset", "double u = uc + (a ? 0.5 : -0.5) / N, v = vc + (b ? 0.5 : -0.5) / N;",
     "double u = uc + (a ? 0.5 : -0.25) / N, v = vc + (b ? 0.5 : -0.5) / N;"),
    ("naive mip weight", "out[texel_index(Nc, face, p, q) + ch] = 0.25 * acc;",
     "out[texel_index(Nc, face, p, q) + ch] = 0.3 * acc;"),
    ("mesh: first instead of farthest hit", "t >= 0.0 && t > best) best = t;",
     "t >= 0.0 && (best == 0.0 || t < best)) best = t;"),
    ("mesh barycentric bound", "a + b <= 1.0 + tol", "a + b <= 1.2 + tol"),
]


def run_mutant(args):
    name, old, new, tmp = args
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, f"{name}: the text to mutate must occur once"
    tag = "".join(ch if ch.isalnum() else "_" for ch in name)
    c_path, so_path = os.path.join(tmp, tag + ".c"), os.path.join(tmp, tag + ".so")
    with open(c_path, "w") as f:
        f.write(src.replace(old, new))
    flags = [f for f in oracle.CFLAGS if f != "-O2"]
    subprocess.check_call(["gcc", "-O1", *flags, "-o", so_path, c_path, "-lm"])
    env = dict(os.environ, SHM_ORACLE_LIB=so_path, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", PINS], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=600)
    failed = [line for line in (r.stdout + r.stderr).splitlines() if line.startswith("FAILED")]
    return name, r.returncode, failed[:1]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    jobs = [(n, o, w, str(tmp_path)) for n, o, w in MUTANTS]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(run_mutant, jobs))
    survivors = [name for name, rc, _ in results if rc == 0]
    for name, rc, failed in results:
        print(f"{name:38s} rc={rc} {failed[0] if failed else ''}")
    assert not survivors, f"mutants the pins accept: {survivors}"
