"""The GPU library's HLLD solver and characteristic PPM reconstruction
(paper_2402_05240_amd/csrc/mhd_physics.hpp), compiled for the host, on the
pins of the oracle's that single out their hardest parts: an isolated
rotational discontinuity must come out exactly (Sec. 2.2 Step 3, Miyoshi &
Kusano's solver), and every branch of the PPM limiter must give the interface
values its data fix (Sec. 2.2 Step 6, the Colella-Sekora limiter)."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import ref
from test_oracle_units import (GAM, _cons_from_prim, _ppmc_along_field, _rotational_discontinuity,
                               ppm_branch_cases)

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


@pytest.fixture(scope="module")
def ppm_probe(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("ppm_probe")
    shutil.copy(os.path.join(CSRC, "mhd_physics.hpp"), d / "mhd_physics.hpp")
    shutil.copy(os.path.join(HERE, "physics_check", "ppm_probe.cpp"), d / "ppm_probe.cpp")
    exe = d / "ppm_probe"
    subprocess.run([gxx, "-O1", "-std=c++17", "-ffp-contract=off", "-o", str(exe),
                    str(d / "ppm_probe.cpp")], check=True, cwd=d)

    def run(stencils, bns, gam, primitive=False):
        text = "\n".join(" ".join("%.17g" % x for x in list(np.ravel(st)) + [bn, gam])
                         for st, bn in zip(stencils, bns))
        out = subprocess.run([str(exe), "1" if primitive else "0"], input=text, check=True,
                             capture_output=True, text=True).stdout
        rows = np.array([[float(x) for x in line.split()] for line in out.strip().splitlines()])
        return rows[:, :7], rows[:, 7:]
    return run


@pytest.mark.parametrize("primitive", [False, True])
def test_device_ppm_limiter_branches(ppm_probe, primitive):
    """The oracle's branch-by-branch PPM pins, on the device header: PPMC along
    one characteristic field, PPMP along one primitive."""
    def one(sten, bn, gam):
        fm, fp = ppm_probe([sten], [bn], gam, primitive=primitive)
        return fm[0], fp[0]
    for q, (s, em, ep) in enumerate(ppm_branch_cases()):
        _ppmc_along_field(s, em, ep, seed=80 + q, reps=8, ppmc=one, primitive=primitive)


@pytest.mark.parametrize("primitive", [False, True])
def test_device_ppm_equals_oracle_on_random_stencils(ppm_probe, primitive):
    """Same reconstruction, same readings: the device header's PPMC (PPMP) and
    the oracle's agree to rounding on random five-cell stencils, smooth ones
    and ones with a jump, so that every limiter branch is taken."""
    rng = np.random.default_rng(46 + int(primitive))
    stencils, bns = [], []
    for _ in range(400):
        W = np.array([rng.uniform(0.3, 3.0), *rng.normal(0, 1, 3), rng.uniform(0.1, 3.0),
                      *rng.normal(0, 1, 2)])
        if rng.uniform() < 0.5:
            d = rng.normal(0, 0.05, 7) * np.abs(W).clip(0.1)
            c = rng.normal(0, 1, 3)
            sten = np.stack([W + (c[0] * j + c[1] * j * j + c[2] * j ** 3 / 4) * d
                             for j in range(-2, 3)])
        else:
            jump = rng.normal(0, 0.3, 7) * np.abs(W).clip(0.1)
            k = int(rng.integers(1, 5))
            sten = np.stack([W * (1 + rng.normal(0, 0.02, 7)) + (jump if j >= k else 0)
                             for j in range(5)])
        sten[:, 0] = np.abs(sten[:, 0]) + 0.05
        sten[:, 4] = np.abs(sten[:, 4]) + 0.05
        stencils.append(sten)
        bns.append(rng.normal(0, 1))
    fm, fp = ppm_probe(stencils, bns, GAM, primitive=primitive)
    fn = ref.ppmp if primitive else ref.ppmc
    for q, (sten, bn) in enumerate(zip(stencils, bns)):
        om, op = fn(sten, bn, GAM)
        tol = 1e-12 * (np.abs(sten).max() + 1.0)
        assert np.abs(fm[q] - om).max() <= tol, q
        assert np.abs(fp[q] - op).max() <= tol, q
