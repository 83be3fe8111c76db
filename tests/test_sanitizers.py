"""CPU builds under the address and undefined-behaviour sanitizers: the FP64
oracle (every entry point, with the brute-force and trajectory-centric
forms compared bit for bit) and the host-side planning of the general-mesh
index.  The sanitizers abort the driver on an out-of-bounds access, a leak,
signed overflow or another undefined operation."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _build_and_run(cmd, exe, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("asan" in r.stderr or "ubsan" in r.stderr):
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr[-3000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
    return run.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    out = _build_and_run(["gcc", "-std=c11", "-fopenmp", "-ffp-contract=off", *SAN,
                          os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe, "-lm"], exe,
                         env={**os.environ, "OMP_NUM_THREADS": "4"})
    assert "oracle driver: ok" in out


def test_host_planning_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_logic_driver")
    out = _build_and_run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_2512_20829_amd", "csrc"),
                          os.path.join(ROOT, "tests", "sanitize", "host_logic_driver.cpp"), "-o", exe], exe)
    assert "host logic driver: ok" in out
