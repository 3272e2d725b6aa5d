"""The complex-step build of the oracle (tests/complex_step): the unchanged
oracle source compiled with a complex-step scalar.  Pins it before the GPU
adjoint tests rely on it: its real part is the oracle's step bit for bit, its
directional derivatives agree with central differences of the real oracle
(to the differences' own accuracy) and are linear in the direction."""
import numpy as np
import pytest

from oracle import ref
from paper_2402_05240_amd import inputs as I
from complex_step import cs


@pytest.fixture(scope="module")
def cso(tmp_path_factory):
    return cs.build(tmp_path_factory.mktemp("cs_oracle"))


def _dir(g, s, seed):
    rng = np.random.default_rng(seed)
    ds = {f: rng.standard_normal(s[f].shape) for f in I.FIELDS}
    I._periodic_face_copy(g, ds)
    return ds


@pytest.mark.parametrize("recon", [I.RECON_PCM, I.RECON_PLMC, I.RECON_PPMC, I.RECON_PLMP])
def test_complex_step_real_part_is_the_oracle(cso, recon):
    g, s = I.turbulence((9, 10, 9), recon=recon)
    dt = ref.cfl_dt(g, s)
    out, _, st = cso.jvp(g, s, _dir(g, s, 1), [dt, 0.9 * dt])
    r1, _, st1 = ref.step(g, s, dt)
    r2, _, st2 = ref.step(g, r1, 0.9 * dt)
    assert st == (st1 | st2)
    for f in I.FIELDS:
        assert np.array_equal(out[f], r2[f]), f


@pytest.mark.parametrize("recon", [I.RECON_PLMC, I.RECON_PCM, I.RECON_PPMC])
def test_complex_step_matches_central_differences(cso, recon):
    g, s = I.turbulence((9, 10, 9), recon=recon)
    dt = ref.cfl_dt(g, s)
    ds = _dir(g, s, 2)
    _, jv, _ = cso.jvp(g, s, ds, [dt])
    h = 1e-7
    p, _, _ = ref.step(g, {f: s[f] + h * ds[f] for f in I.FIELDS}, dt)
    m, _, _ = ref.step(g, {f: s[f] - h * ds[f] for f in I.FIELDS}, dt)
    for f in I.FIELDS:
        fd = (p[f] - m[f]) / (2 * h)
        assert np.abs(fd - jv[f]).max() <= 1e-6 * np.abs(jv[f]).max(), f


def test_complex_step_is_linear_in_the_direction(cso):
    g, s = I.turbulence((9, 9, 10))
    dt = ref.cfl_dt(g, s)
    a, b = _dir(g, s, 3), _dir(g, s, 4)
    _, ja, _ = cso.jvp(g, s, a, [dt])
    _, jb, _ = cso.jvp(g, s, b, [dt])
    _, jc, _ = cso.jvp(g, s, {f: 2.0 * a[f] - 3.0 * b[f] for f in I.FIELDS}, [dt])
    for f in I.FIELDS:
        want = 2.0 * ja[f] - 3.0 * jb[f]
        assert np.abs(jc[f] - want).max() <= 1e-13 * np.abs(want).max(), f
