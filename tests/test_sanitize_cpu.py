"""Sanitizer builds of the host code (CPU, no GPU needed): the C oracle with
the address and undefined-behaviour sanitizers, run over every routine on
small seeded inputs; the library's host side (state tables, plan counts, Pade,
argument validation, failure injection, the no-device path) built with the
same sanitizers on the host code only and exercised by a driver.  Any report
aborts the program and fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
                    "-fsanitize=address,undefined",
                    "-o", exe, os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "cos_oracle.c"),
                    "-lm"], check=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=SAN_ENV)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert r.stdout.count("n=") == 7 * 2 * 2


@pytest.mark.slow
def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    csrc = os.path.join(ROOT, "paper_2507_12349_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in ("cos_level.hip", "cos_sub.hip", "cos_kernels.hip", "cos_mc.hip",
                                            "cos_cdet.hip", "cos_static.hip", "libcos.cpp")]
    exe = str(tmp_path / "abi_san")
    # the sanitizers apply to the host code only (each flag right after -Xarch_host)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san,
                    "-I", os.path.join(ROOT, "include"), "-o", exe, os.path.join(HERE, "abi_driver.cpp"), *srcs],
                   check=True, timeout=900, capture_output=True)
    env = dict(SAN_ENV, HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert "host checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
