"""The reverse derivatives of HLLD, the characteristic eigen-system and the
PLMC / PLMP / PPMC / PPMP reconstructions (paper_2402_05240_amd/csrc/mhd_adjoint.hpp),
compiled for the host, against forward-mode dual numbers pushed through the
device physics header itself (tests/adjoint_check/check.cpp): J^T a from
the hand-written reverse code must equal the dual-number Jacobian contracted
with a, over random states that reach every HLLD fan region, B_n = 0,
identical left/right states, B_perp = 0 and all limiter cases."""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2402_05240_amd", "csrc")


def test_reverse_derivatives_match_dual_numbers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    shutil.copy(os.path.join(CSRC, "mhd_physics.hpp"), tmp_path / "mhd_physics.hpp")
    shutil.copy(os.path.join(CSRC, "mhd_adjoint.hpp"), tmp_path / "mhd_adjoint.hpp")
    # the dual instantiation includes the physics a second time, inside its own namespace
    with open(os.path.join(CSRC, "mhd_physics.hpp")) as f:
        body = f.read().replace("#pragma once", "")
    (tmp_path / "phys_copy.hpp").write_text(body)
    shutil.copy(os.path.join(HERE, "adjoint_check", "check.cpp"), tmp_path / "check.cpp")
    exe = tmp_path / "check"
    subprocess.run([gxx, "-O1", "-std=c++17", "-o", str(exe), str(tmp_path / "check.cpp")],
                   check=True, cwd=tmp_path)
    out = subprocess.run([str(exe), "20000"], check=True, capture_output=True, text=True).stdout
    print(out)
    found = re.findall(r"(HLLD|PLMP|PLMC|PPMP|PPMC): worst rel err ([0-9.e+-]+), bad (\d+)", out)
    assert {name for name, _, _ in found} == {"HLLD", "PLMP", "PLMC", "PPMP", "PPMC"}, out
    for name, worst, bad in found:
        assert int(bad) == 0 and float(worst) <= 1e-12, (name, worst, bad)
