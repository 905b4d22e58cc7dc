"""Sanitizer runs on the CPU: the oracle (plain C) built with AddressSanitizer
and UndefinedBehaviorSanitizer runs every oracle pin, and the library built
with the same sanitizers on its host code (the device code is the ordinary
gfx950 build) runs every host-side argument check of the C ABI.  No out-of-
bounds access, use after free or undefined arithmetic on those paths.  Each
run is a child Python process with the instrumented build loaded in place of
the ordinary one and the sanitizer runtime preloaded."""
import os
import subprocess
import sys

import pytest

import oracle
import paper_2602_20063_amd as shm
from paper_2602_20063_amd import build as shm_build
from conftest import ROOT

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def runtime(compiler, name):
    path = subprocess.run([compiler, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{compiler} has no {name}")
    return path


def run_child(env, args, timeout):
    r = subprocess.run([sys.executable, *args], cwd=ROOT, env=dict(os.environ, **SAN_ENV, **env),
                       capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "shm_oracle_san.so")
    flags = [f for f in oracle.CFLAGS if f != "-O2"]
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", *flags, "-o", lib, oracle._SRC, "-lm"])
    env = {"LD_PRELOAD": runtime("gcc", "libasan.so"), "SHM_ORACLE_LIB": lib}
    out = run_child(env, ["-c", "import ctypes, oracle; assert oracle.lib()._name == %r; "
                                "ctypes.CDLL(None).__asan_init; print('instrumented oracle loaded')" % lib], 120)
    assert "instrumented oracle loaded" in out
    out = run_child(env, ["-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_pins.py")], 900)
    assert " passed" in out and "failed" not in out


def test_abi_checks_under_asan_and_ubsan(tmp_path):
    objs, procs = [], []
    for src in shm_build.sources():
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = ["hipcc", *[f for f in shm_build.FLAGS if f != "-shared"], "-g",
               "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
               "-Xarch_host", "-fsanitize=undefined", "-c", src, "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    for p in procs:
        out, _ = p.communicate()
        assert p.returncode == 0, out.decode(errors="replace")[-3000:]
    lib = str(tmp_path / "libshm_san.so")
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined", "-o", lib, *objs])
    env = {"LD_PRELOAD": runtime("hipcc", "libclang_rt.asan-x86_64.so"), "SHM_LIBRARY": lib}
    out = run_child(env, ["-c", "import ctypes, paper_2602_20063_amd as s; assert s.lib()._name == %r; "
                                "ctypes.CDLL(None).__asan_init; print('instrumented library loaded')" % lib], 300)
    assert "instrumented library loaded" in out
    out = run_child(env, ["-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider", "-m", "not gpu",
                          os.path.join(ROOT, "tests", "test_abi.py")], 900)
    assert " passed" in out and "failed" not in out
    assert shm.lib()._name != lib  # this process keeps the ordinary build


def test_planted_out_of_bounds_read_is_reported(tmp_path):
    """Negative control: a copy of the oracle whose corner gather reads one
    texel row and column too far is built the same way; ASan reports a
    heap-buffer overflow in that gather on the first pin that reaches it."""
    src = open(oracle._SRC).read()
    good = "lut + texel_index(N, face, i0 + i, j0 + j)"
    assert src.count(good) == 1
    bad = tmp_path / "shm_oracle_planted.c"
    bad.write_text(src.replace(good, "lut + texel_index(N, face, i0 + i + 1, j0 + j + 1)"))
    lib = str(tmp_path / "planted.so")
    flags = [f for f in oracle.CFLAGS if f != "-O2"]
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", *flags, "-o", lib, str(bad), "-lm"])
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=runtime("gcc", "libasan.so"), SHM_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode != 0
    assert "ERROR: AddressSanitizer: heap-buffer-overflow" in out and "gather_corners" in out, out[-3000:]
