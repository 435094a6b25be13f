"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The C oracle is rebuilt with gcc's -fsanitize=address,undefined and its
  pins (test_oracle_pins.py, test_oracle_regex.py, without the two
  multi-second full-size cases) run again on it in a child process.
* The library's host objects (parem_api.cpp: validation, completion of
  partial tables, speculated sets, every table layout; parem_regex.cpp: the
  regular-expression front-end) are rebuilt with the sanitizers on the host
  side only and linked with the other objects of the normal build;
  sanitize_host.py drives them in a child process (no GPU is needed: a
  compile ends in PAREM_EDEVICE after all host work).

Any sanitizer report fails the child (halt_on_error, no recovery)."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(cmd, env, timeout):
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, out
    return r


def test_oracle_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip() \
        if gcc else ""
    if not gcc or not os.path.isabs(asan):
        pytest.skip("gcc with libasan is not available")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", lib,
                           os.path.join(ROOT, "oracle", "parem_oracle.c")])
    env = dict(os.environ, PAREM_ORACLE_LIB=lib, LD_PRELOAD=asan, **SAN_ENV)
    r = _run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
              "-k", "not u64_wide and not full_size", "tests/test_oracle_pins.py", "tests/test_oracle_regex.py"],
             env, 900)
    assert " passed" in r.stdout


def test_host_compile_path_under_asan_and_ubsan(tmp_path):
    from paper_1412_1741_amd import build as B

    runtimes = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not runtimes or not os.path.exists(B.hipcc()):
        pytest.skip("hipcc or its AddressSanitizer runtime is not available")
    others = [os.path.join(B.OBJ, s + ".o") for s in B.SOURCES if s not in ("parem_api.cpp", "parem_regex.cpp")]
    if not all(os.path.exists(o) for o in others):
        pytest.skip("the library's objects are not built (python -m paper_1412_1741_amd.build)")
    san = ["-O1", "-g"] + [f for flag in ("-fsanitize=address", "-fsanitize=undefined",
                                          "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer")
                           for f in ("-Xarch_host", flag)]
    objs = []
    for src in ("parem_api.cpp", "parem_regex.cpp"):
        obj = str(tmp_path / (src + ".o"))
        flags = [f for f in B.HIP_FLAGS if f not in ("-O3", "-Wall")]
        subprocess.check_call([B.hipcc(), *flags, *san, "-I", os.path.join(ROOT, "include"), "-c",
                               os.path.join(B.CSRC, src), "-o", obj], stderr=subprocess.DEVNULL)
        objs.append(obj)
    lib = str(tmp_path / "libparem_san.so")
    subprocess.check_call([B.hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs, *others])
    env = dict(os.environ, LD_PRELOAD=runtimes[-1], **SAN_ENV)
    r = _run([sys.executable, os.path.join(ROOT, "tests", "sanitize_host.py"), lib], env, 900)
    assert "host paths done" in r.stdout
