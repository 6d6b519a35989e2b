"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle and the host side of the library (planning of every kind, shaped
trees' node tables, batch planning, Huffman codes, argument checks) are
compiled with both sanitizers and driven over edge cases by the programs in
tests/native/; a sanitizer report or an unexpected return code fails the test.
Device code is compiled as usual (the sanitizer flags apply to the host pass
only) and is never run here."""
import glob
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
NATIVE = os.path.join(HERE, "native")
CSRC = os.path.join(ROOT, "paper_1610_03524_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:halt_on_error=1",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-fno-sanitize-recover=undefined", "-o", exe, os.path.join(NATIVE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "wavelet_oracle.c")])
    r = _run([exe], env=dict(os.environ, **SAN_ENV), timeout=300)
    assert "all calls returned the expected codes" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


def test_library_host_code_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    procs, objs = [], []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *flags, "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for src, p in zip(srcs, procs):
        out, err = p.communicate(timeout=600)
        assert p.returncode == 0, f"{src}\n{err}"
    drv = str(tmp_path / "plan_driver.o")
    _run([HIPCC, "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
          "-x", "c++", "-c", os.path.join(NATIVE, "plan_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "plan_driver")
    _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
          "-fsanitize=undefined", "-o", exe, drv, *objs, "-L/opt/rocm/lib", "-lamdhip64"])
    env = dict(os.environ, **SAN_ENV)
    env["LD_LIBRARY_PATH"] = "/opt/rocm/lib:" + env.get("LD_LIBRARY_PATH", "")
    r = _run([exe], env=env, timeout=300)
    assert "every call returned an allowed code" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
