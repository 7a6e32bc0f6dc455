"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (oracle.c) built with -fsanitize=address,undefined, loaded into a
  child Python with the sanitizer runtimes preloaded, runs the whole pin suite
  (tests/test_oracle_pins.py).
* The library's host planner (capi.hip's host code, sanitized through
  -Xarch_host; the kernels' objects as built) linked into tests/asan_planner.cpp,
  which drives validation, the Table 1 block arithmetic and the argument checks
  of every entry point without reaching a HIP call.
* A planted heap overflow and a planted array-bounds error, built and loaded
  the same way as the oracle, are reported: the harness itself is live.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def gcc_runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                          check=True).stdout.strip()


def preload_env(extra=None):
    env = dict(os.environ, **SAN_ENV)
    env["LD_PRELOAD"] = gcc_runtime("libasan.so") + ":" + gcc_runtime("libubsan.so")
    env["OMP_NUM_THREADS"] = "4"
    env.update(extra or {})
    return env


@pytest.mark.parametrize("san,body,report", [
    # heap overflow, in a build with AddressSanitizer alone
    ("address", "int *a = malloc(4 * sizeof(int)); volatile int *p = a; p[i] = 7; int r = p[0]; free(a); return r;",
     "AddressSanitizer"),
    # index past a fixed-size array: UndefinedBehaviorSanitizer's bounds check
    ("address,undefined", "int a[4] = {0, 1, 2, 3}; a[i] = 7; return a[0];", "runtime error"),
], ids=["asan", "ubsan"])
def test_planted_error_is_reported(tmp_path, san, body, report):
    src = tmp_path / "bad.c"
    src.write_text("#include <stdlib.h>\nint poke(int i) { " + body + " }\n")
    lib = tmp_path / "libbad.so"
    subprocess.run(["gcc", "-O1", "-g", "-fsanitize=" + san, "-fno-sanitize-recover=all",
                    "-fPIC", "-shared", "-o", str(lib), str(src)], check=True)
    code = f"import ctypes; ctypes.CDLL({str(lib)!r}).poke(9)"
    r = subprocess.run([sys.executable, "-c", code], env=preload_env(), capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert report in r.stderr, r.stderr[-2000:]


def test_oracle_pins_under_asan_ubsan(tmp_path):
    import oracle

    lib = oracle.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-q",
                        "-x", "-p", "no:cacheprovider"], cwd=ROOT, env=preload_env({"ORACLE_LIB": lib}),
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    assert " passed" in out


def test_host_planner_under_asan_ubsan(tmp_path):
    from paper_1905_02803_amd import build

    bdir = os.path.join(build.HERE, "_build")
    objs = [os.path.join(bdir, n.replace(".hip", ".o")) for n in build.SOURCES if n != "capi.hip"]
    if not all(os.path.exists(o) for o in objs):
        build.build()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", build.CSRC]
    capi = str(tmp_path / "capi_asan.o")
    # the host pass of capi.hip instrumented; its device pass (none used here) as usual
    subprocess.run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-omit-frame-pointer"] + inc +
                   ["-c", os.path.join(build.CSRC, "capi.hip"), "-o", capi], check=True, capture_output=True)
    drv = str(tmp_path / "driver.o")
    subprocess.run([CLANGXX, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "asan_planner.cpp"),
                    "-o", drv], check=True)
    exe = str(tmp_path / "planner")
    subprocess.run([CLANGXX, "-fsanitize=address,undefined", drv, capi] + objs +
                   ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe], check=True)
    r = subprocess.run([exe], env=dict(os.environ, **SAN_ENV), capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    assert "0 failures" in r.stdout
