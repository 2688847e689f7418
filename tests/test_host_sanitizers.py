"""Host sanitizer builds (no GPU needed).

* The oracle (oracle/mfm_oracle.c), serial and OpenMP, under AddressSanitizer
  and UndefinedBehaviorSanitizer: every exported stage on small periodic and
  open sets, both schemes, the optional limiters, the levelled fluxes, and its
  error returns (tests/sanitize/oracle_driver.c).
* The library's host code (csrc/api.hip: parameter, argument, capacity and
  call-order checks, context creation and its error path) built with the
  same sanitizers on the host side only (device code untouched), driven by
  tests/sanitize/abi_driver.cpp through the C ABI with calls that all return
  before any launch.  Without a GPU, context creation fails at its first
  allocation and the partly built context's clean-up is what runs.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
ASAN_ENV = {"ASAN_OPTIONS": "abort_on_error=0:halt_on_error=1:detect_leaks=1",
            "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(cmd, env=None, timeout=300):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run(cmd, capture_output=True, text=True, env=e, timeout=timeout)


def _clean(r):
    out = r.stdout + r.stderr
    # a sanitizer report names its sanitizer (UBSan in its summary line)
    for tag in ("AddressSanitizer", "UndefinedBehaviorSanitizer", "LeakSanitizer", ": runtime error:"):
        assert tag not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


@pytest.mark.parametrize("openmp", [False, True])
def test_oracle_under_asan_and_ubsan(tmp_path, openmp):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_asan")
    cmd = [gcc, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-o", exe, os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "mfm_oracle.c"), "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    r = _run(cmd)
    assert r.returncode == 0, r.stderr
    out = _clean(_run([exe], env=dict(ASAN_ENV, OMP_NUM_THREADS="4")))
    assert "lone particle: rc=-5" in out and out.count("rc=0") == 3, out


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not found")
    from paper_1712_01294_amd import build as B
    csrc = B.CSRC
    # host code of api.hip instrumented; the other sources as the library builds them
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in B.SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        flags = [f for f in B.FLAGS if f != "-O3"] + ["-O1", "-g"] + (san if src == "api.hip" else [])
        r = _run([hipcc, *flags, "-c", os.path.join(csrc, src), "-o", obj])
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    lib = str(tmp_path / "libmfm_san.so")
    r = _run([clang, "-shared", "-fsanitize=address,undefined", "-o", lib, *objs, "-L/opt/rocm/lib",
              "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "abi_asan")
    r = _run([clang, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-o", exe,
              os.path.join(SAN, "abi_driver.cpp"), lib, "-Wl,-rpath," + str(tmp_path)])
    assert r.returncode == 0, r.stderr[-3000:]
    out = _clean(_run([exe], env=ASAN_ENV))
    assert "0 unexpected results" in out, out
