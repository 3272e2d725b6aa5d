"""Sanitizer builds of the host code (no GPU): the oracle, the host build of
the device physics with its hand-written reverse derivatives (the adjoint
check harness) and the HLLD probe, compiled with AddressSanitizer and
UndefinedBehaviorSanitizer, every error fatal; each program must run clean.
The oracle's driver (tests/sanitize/oracle_driver.c) steps every
reconstruction on small ragged grids with periodic, outflow and mixed
boundaries and calls each unit entry point."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2402_05240_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _need(tool):
    path = shutil.which(tool)
    if path is None:
        pytest.skip("no %s" % tool)
    return path


def _run(exe, *args):
    r = subprocess.run([str(exe)] + list(args), capture_output=True, text=True, env=ENV,
                       timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, \
        r.stderr[-4000:]
    return r.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    gcc = _need("gcc")
    exe = tmp_path / "oracle_san"
    subprocess.run([gcc, "-std=c11", "-O1", "-ffp-contract=off", "-fno-fast-math"] + SAN +
                   ["-I", os.path.join(ROOT, "oracle"), "-o", str(exe),
                    os.path.join(ROOT, "oracle", "vlct_ref.c"),
                    os.path.join(HERE, "sanitize", "oracle_driver.c"), "-lm"], check=True)
    out = _run(exe)
    assert "0 failures" in out, out


def test_adjoint_harness_under_asan_ubsan(tmp_path):
    gxx = _need("g++")
    shutil.copy(os.path.join(CSRC, "mhd_physics.hpp"), tmp_path / "mhd_physics.hpp")
    shutil.copy(os.path.join(CSRC, "mhd_adjoint.hpp"), tmp_path / "mhd_adjoint.hpp")
    with open(os.path.join(CSRC, "mhd_physics.hpp")) as f:
        (tmp_path / "phys_copy.hpp").write_text(f.read().replace("#pragma once", ""))
    shutil.copy(os.path.join(HERE, "adjoint_check", "check.cpp"), tmp_path / "check.cpp")
    exe = tmp_path / "check_san"
    subprocess.run([gxx, "-O1", "-std=c++17"] + SAN + ["-o", str(exe), str(tmp_path / "check.cpp")],
                   check=True, cwd=tmp_path)
    out = _run(exe, "2000")
    assert "HLLD" in out and "PPMC" in out, out


def test_hlld_probe_under_asan_ubsan(tmp_path):
    gxx = _need("g++")
    shutil.copy(os.path.join(CSRC, "mhd_physics.hpp"), tmp_path / "mhd_physics.hpp")
    shutil.copy(os.path.join(HERE, "physics_check", "hlld_probe.cpp"), tmp_path / "hlld_probe.cpp")
    exe = tmp_path / "probe_san"
    subprocess.run([gxx, "-O1", "-std=c++17"] + SAN + ["-o", str(exe),
                    str(tmp_path / "hlld_probe.cpp")], check=True, cwd=tmp_path)
    line = " ".join(["1.0 0.3 -0.2 0.1 0.6 0.4 -0.3", "0.5 -0.4 0.2 0.0 0.3 -0.1 0.2", "0.8",
                     "1.6666666666666667"])
    r = subprocess.run([str(exe)], input=line + "\n", capture_output=True, text=True, env=ENV,
                       timeout=60)
    assert r.returncode == 0 and "runtime error" not in r.stderr, r.stderr[-2000:]
    assert len(r.stdout.split()) == 8
