"""AddressSanitizer and UndefinedBehaviorSanitizer over host code (CPU only).

Two builds made here, into a temporary directory, and exercised by the
existing CPU tests in a child interpreter that preloads the sanitizer
runtimes:
* the oracle (plain C, gcc -fsanitize=address,undefined), under its pins;
* the library's host code -- instance validation and re-layout, workspace
  sizing, layout queries, error paths -- with the sanitizers on the host
  side only (device code is compiled as usual and never runs here), under
  the ABI tests.
Any sanitizer report aborts the child (halt_on_error / no recovery) and
fails the test."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    if out.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not available")
    return path


def _clang_runtime():
    """The shared AddressSanitizer runtime of hipcc's clang (it carries the
    UBSan handlers too)."""
    clang = os.path.join(os.path.dirname(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")), "..", "llvm", "bin",
                         "clang")
    out = subprocess.run([clang, "--print-resource-dir"], capture_output=True, text=True)
    path = os.path.join(out.stdout.strip(), "lib", "linux", "libclang_rt.asan-x86_64.so")
    if out.returncode != 0 or not os.path.exists(path):
        pytest.skip("clang's sanitizer runtime not available")
    return path


def _child(tests, env_extra, tmp_path, k=None, preload=None):
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = preload or (_runtime("libasan.so") + ":" + _runtime("libubsan.so"))
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + tests
    if k:
        cmd += ["-k", k]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    text = res.stdout + res.stderr
    assert res.returncode == 0 and "ERROR: AddressSanitizer" not in text and "runtime error:" not in text, \
        text[-4000:]
    return text


def test_oracle_under_asan_ubsan(tmp_path):
    lib = tmp_path / "libtdpt_oracle_asan.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-fPIC", "-shared", "-o", str(lib),
                           os.path.join(ROOT, "oracle", "tdpt_oracle.c"), "-lm"])
    syms = subprocess.run(["nm", "-D", str(lib)], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms
    _child(["tests/test_oracle_pins.py", "tests/test_constraints.py", "tests/test_adaptive.py"],
           {"TDPT_ORACLE_LIB": str(lib)}, tmp_path,
           k="not long_run and not four_by_four and not positions_sample")


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2506_14781_amd import build as B
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    lib = tmp_path / "libtdpt_asan.so"
    flags = [f for f in B.HIPCC_FLAGS if f != "-O3"] + ["-O1", "-g", "-fno-omit-frame-pointer"]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined"]
    cmd = [hipcc] + flags + san + ["-I", B.INCLUDE, "-I", B.CSRC, "-o", str(lib)] + \
        [os.path.join(B.CSRC, s) for s in B.SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    syms = subprocess.run(["nm", "-D", str(lib)], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms  # the host code is instrumented
    _child(["tests/test_abi.py"], {"TDPT_LIB": str(lib)}, tmp_path, k="not missing_library",
           preload=_clang_runtime())
