"""The GPU library's HLLD solver (paper_2402_05240_amd/csrc/mhd_physics.hpp),
compiled for the host, on the pins of the oracle's solver that single out
its double-star (Alfven) states: an isolated rotational discontinuity must
come out exactly (Sec. 2.2 Step 3, Miyoshi & Kusano's solver)."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import ref
from test_oracle_units import GAM, _cons_from_prim, _rotational_discontinuity

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2402_05240_amd", "csrc")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("hlld_probe")
    shutil.copy(os.path.join(CSRC, "mhd_physics.hpp"), d / "mhd_physics.hpp")
    shutil.copy(os.path.join(HERE, "physics_check", "hlld_probe.cpp"), d / "hlld_probe.cpp")
    exe = d / "hlld_probe"
    subprocess.run([gxx, "-O1", "-std=c++17", "-ffp-contract=off", "-o", str(exe),
                    str(d / "hlld_probe.cpp")], check=True, cwd=d)

    def run(cases):
        text = "\n".join(" ".join("%.17g" % x for x in list(wl) + list(wr) + [bn, gam])
                         for wl, wr, bn, gam in cases)
        out = subprocess.run([str(exe)], input=text, check=True, capture_output=True,
                             text=True).stdout
        return np.array([[float(x) for x in line.split()] for line in out.strip().splitlines()])
    return run


@pytest.mark.parametrize("left_wave", [True, False])
def test_device_hlld_resolves_isolated_rotational_discontinuity(probe, left_wave):
    rng = np.random.default_rng(32)
    cases, expect, scales = [], [], []
    for _ in range(200):
        rho, p = rng.uniform(0.3, 3.0), rng.uniform(0.1, 2.0)
        bn = rng.choice([-1.0, 1.0]) * rng.uniform(0.3, 2.0)
        bt = rng.uniform(0.2, 2.0)
        phi_l = rng.uniform(0, 2 * np.pi)
        phi_r = phi_l + rng.uniform(0.3, np.pi)
        v0 = rng.uniform(-1.0, 1.0, 2)
        lab = (-0.3 if left_wave else 0.3) * abs(bn) / math.sqrt(rho)
        Wl, Wr, ca = _rotational_discontinuity(rho, p, bn, bt, phi_l, phi_r, v0, lab, left_wave)
        cases.append((Wl, Wr, bn, GAM))
        fe = ref.phys_flux(Wr if left_wave else Wl, bn, GAM)
        expect.append(fe)
        Ul, Ur = _cons_from_prim(Wl, bn), _cons_from_prim(Wr, bn)
        scales.append(np.abs(fe).max() + np.abs(Ur - Ul).max() * ca)
    out = probe(cases)
    f = out[:, :7]
    err = np.abs(f - np.array(expect)).max(axis=1) / np.array(scales)
    assert err.max() <= 1e-13, err.max()
    # the discontinuity is not at the contact: the upwind side is the flow's
    assert np.all(out[:, 7] == (1.0 if left_wave else -1.0))


def test_device_hlld_equals_oracle_on_random_states(probe):
    """Same solver, same readings: the host build of the device header and the
    oracle agree to rounding on random pairs of states over every fan region."""
    rng = np.random.default_rng(33)
    cases = []
    for _ in range(500):
        def w():
            return np.array([rng.uniform(0.2, 3.0), rng.uniform(-3, 3), rng.uniform(-2, 2),
                             rng.uniform(-2, 2), rng.uniform(0.05, 3.0), rng.uniform(-2, 2),
                             rng.uniform(-2, 2)])
        cases.append((w(), w(), rng.uniform(-2, 2), GAM))
    out = probe(cases)
    for (wl, wr, bn, gam), row in zip(cases, out):
        fo = ref.hlld(wl, wr, bn, gam)
        assert np.abs(row[:7] - fo).max() <= 1e-12 * (np.abs(fo).max() + 1.0)
