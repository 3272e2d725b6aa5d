"""Adjoint of one step on the GPU (vlct_step_adjoint) against the oracle.

For a step of fixed size dt, out = S(in), and the adjoint returns
lam_in = (dS/d in)^T lam_out.  The adjoint identity
    <lam_in, delta> = <lam_out, (dS/d in) delta>
is checked with the right side from central differences of the oracle's step
along delta: per input coordinate on a small grid (each is one element of
lam_in; every field, sampled coordinates) and along random directions on a
larger grid.  The step is only piecewise smooth (limiters, HLLD regions, CT
upwinding): a coordinate whose difference quotients at two step sizes
disagree has a branch boundary within the difference stencil and is not
compared; at most a small fraction may be skipped."""
import numpy as np
import pytest

from oracle import ref
from paper_2402_05240_amd import inputs as I
from parity_util import FIELDS, gpu_available

pytestmark = pytest.mark.gpu

RECONS = [I.RECON_PCM, I.RECON_PLMC, I.RECON_PLMP, I.RECON_PPMC, I.RECON_PPMP]
# tolerances relative to sum |lam_out * d out|, the size of the compared
# products: the central differences carry ~1e-16 / H rounding per output
# element (a few 1e-9 for single coordinates, ~1e-11 along full directions)
TOL_SMOOTH = 1e-6   # difference quotients at H and H/4 closer than this: no branch boundary
TOL_ELEM = 1e-7
TOL_DIR = 1e-8
H = 1e-6            # central-difference step for O(1) state values


def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _say(msg):
    print(msg, flush=True)


def _state(n, recon, seed):
    """Turbulence (Gaussian random velocity, B = B_x0 + curl A) with smooth
    density and pressure variations added, so that every term of the flux
    Jacobians is exercised."""
    g, s = I.turbulence(n, recon=recon, seed_v=seed, seed_a=seed + 1)
    rng = np.random.default_rng(seed + 2)
    x, y, z = I._centres(g)
    ph = rng.uniform(0.0, 2.0 * np.pi, 4)
    fr = 1.0 + 0.3 * np.sin(2 * np.pi * x + ph[0]) * np.cos(2 * np.pi * (y + z) + ph[1])
    fp = 1.0 + 0.25 * np.cos(2 * np.pi * (x - y) + ph[2]) * np.sin(2 * np.pi * z + ph[3])
    v = [s[m] / s["rho"] for m in ("mx", "my", "mz")]
    rho = s["rho"] * fr
    s["rho"] = rho
    for m, vv in zip(("mx", "my", "mz"), v):
        s[m] = rho * vv
    s["E"] = I._cell_energy(g, rho, v[0], v[1], v[2], fp / g.gamma, s["bx"], s["by"], s["bz"])
    return g, s


def _random_cotangent(g, seed):
    rng = np.random.default_rng(seed)
    return {f: rng.standard_normal(g.field_shape(f)) for f in FIELDS}


def _dup(g, f, idx):
    """The periodic duplicate of a face on plane 0 (it moves with the face)."""
    k, j, i = idx
    if f == "bx" and i == 0:
        return (k, j, g.nx)
    if f == "by" and j == 0:
        return (k, g.ny, i)
    if f == "bz" and k == 0:
        return (g.nz, j, i)
    return None


def _fd(g, s, dt, lam, delta, h):
    """Central difference of <lam, S(s)> along delta: (value, scale)."""
    outs = []
    for sign in (1.0, -1.0):
        t = {f: s[f] + sign * h * delta[f] for f in FIELDS}
        out, _, st = ref.step(g, t, dt, nthreads=4)
        assert st == 0
        outs.append(out)
    d = {f: (outs[0][f] - outs[1][f]) / (2.0 * h) for f in FIELDS}
    val = sum(float(np.sum(lam[f] * d[f])) for f in FIELDS)
    scale = sum(float(np.sum(np.abs(lam[f] * d[f]))) for f in FIELDS)
    return val, scale


def _unit(g, f, idx):
    delta = {q: np.zeros(g.field_shape(q)) for q in FIELDS}
    delta[f][idx] = 1.0
    dup = _dup(g, f, idx)
    if dup is not None:
        delta[f][dup] = 1.0
    return delta


def _gpu_vjp(g, s, lam, dt):
    from paper_2402_05240_amd.device import Adjoint
    import torch
    adj = Adjoint(g)
    out = adj.vjp(s, lam, dt)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("recon", RECONS)
def test_adjoint_elements_match_oracle_differences(recon):
    """lam_in element by element on a 9 x 10 x 9 periodic grid: 24 sampled
    coordinates of each of the 8 fields (faces on the periodic plane 0
    included), each against a central difference of the oracle's step."""
    _need_gpu()
    g, s = _state((9, 10, 9), recon, 11)
    dt = ref.cfl_dt(g, s)
    lam = _random_cotangent(g, 5)
    _say("adjoint elements: recon %d, grid %s, dt %.3e" % (recon, (g.nx, g.ny, g.nz), dt))
    lin = _gpu_vjp(g, s, lam, dt)
    # the step never reads the input's duplicate faces
    assert not np.any(lin["bx"][:, :, -1]) and not np.any(lin["by"][:, -1, :])
    assert not np.any(lin["bz"][-1])
    rng = np.random.default_rng(17 + recon)
    checked = skipped = 0
    worst = 0.0
    for f in FIELDS:
        shape = list(g.field_shape(f))
        # coordinates of the stored field without the duplicate plane
        if f == "bx":
            shape[2] -= 1
        elif f == "by":
            shape[1] -= 1
        elif f == "bz":
            shape[0] -= 1
        picks = [tuple(int(rng.integers(0, m)) for m in shape) for _ in range(22)]
        # two coordinates on the periodic plane 0 of the face field (or corners of cells)
        picks += [(0, 0, 0), (shape[0] - 1, 0, shape[2] - 1) if f != "bx" else (1, 2, 0)]
        for idx in picks:
            delta = _unit(g, f, idx)
            v1, sc = _fd(g, s, dt, lam, delta, H)
            v2, _ = _fd(g, s, dt, lam, delta, H / 4)
            if abs(v1 - v2) > TOL_SMOOTH * sc:
                skipped += 1
                continue
            got = float(lin[f][idx])
            err = abs(got - v1) / sc
            worst = max(worst, err)
            checked += 1
            assert err <= TOL_ELEM, (f, idx, got, v1, sc)
    _say("checked %d, skipped %d (branch boundary), worst rel err %.2e"
         % (checked, skipped, worst))
    assert skipped <= 0.05 * (checked + skipped)


@pytest.mark.parametrize("recon", RECONS)
def test_adjoint_directional_derivatives(recon):
    """<lam_in, delta> for random directions delta over every coordinate of a
    16 x 12 x 10 grid against central differences of the oracle's step."""
    _need_gpu()
    g, s = _state((16, 12, 10), recon, 23)
    dt = ref.cfl_dt(g, s)
    lam = _random_cotangent(g, 6)
    lin = _gpu_vjp(g, s, lam, dt)
    rng = np.random.default_rng(29)
    for rep in range(3):
        delta = {f: rng.standard_normal(g.field_shape(f)) for f in FIELDS}
        I._periodic_face_copy(g, delta)
        got = sum(float(np.sum(lin[f] * delta[f])) for f in FIELDS)
        errs = []
        for h in (1e-7, 2.5e-8):
            v, sc = _fd(g, s, dt, lam, delta, h)
            errs.append(abs(got - v) / sc)
        _say("recon %d direction %d: <lam_in, delta> = %.12e, rel err %s"
             % (recon, rep, got, ["%.1e" % e for e in errs]))
        assert min(errs) <= TOL_DIR, errs


def test_adjoint_zero_step_is_the_identity():
    """dt = 0: the step is the identity on cells and faces 0..n-1, the output's
    duplicate face copies face 0, so lam_in is lam_out with each duplicate
    face's cotangent moved onto face 0 -- exactly."""
    _need_gpu()
    g, s = _state((9, 9, 11), I.RECON_PLMC, 3)
    lam = _random_cotangent(g, 8)
    lin = _gpu_vjp(g, s, lam, 0.0)
    want = {f: lam[f].copy() for f in FIELDS}
    want["bx"][:, :, 0] += want["bx"][:, :, -1]
    want["bx"][:, :, -1] = 0.0
    want["by"][:, 0, :] += want["by"][:, -1, :]
    want["by"][:, -1, :] = 0.0
    want["bz"][0] += want["bz"][-1]
    want["bz"][-1] = 0.0
    for f in FIELDS:
        assert np.array_equal(lin[f], want[f]), f


def test_adjoint_is_linear_in_the_cotangent():
    _need_gpu()
    g, s = _state((12, 9, 10), I.RECON_PLMC, 31)
    dt = ref.cfl_dt(g, s)
    l1, l2 = _random_cotangent(g, 1), _random_cotangent(g, 2)
    mix = {f: 2.0 * l1[f] - 3.0 * l2[f] for f in FIELDS}
    a, b, c = (_gpu_vjp(g, s, lam, dt) for lam in (l1, l2, mix))
    for f in FIELDS:
        ref_v = 2.0 * a[f] - 3.0 * b[f]
        scale = float(np.abs(2.0 * a[f]).max() + np.abs(3.0 * b[f]).max())
        assert float(np.abs(c[f] - ref_v).max()) <= 1e-13 * scale, f


@pytest.fixture(scope="module")
def cso(tmp_path_factory):
    from complex_step import cs
    return cs.build(tmp_path_factory.mktemp("cs_oracle"))


@pytest.mark.parametrize("recon", RECONS)
def test_adjoint_against_complex_step_of_the_oracle(cso, recon):
    """<lam_in, delta> against <lam_out, J delta> with J delta from the
    complex-step build of the oracle (exact to rounding, every branch at the
    unperturbed state like the adjoint's), for full random directions over
    every coordinate of a 16^3 grid, and lam_in element by element for
    sampled coordinates (J e_j): within 1e-10."""
    _need_gpu()
    g, s = _state((16, 16, 16), recon, 41)
    dt = ref.cfl_dt(g, s)
    lam = _random_cotangent(g, 42)
    lin = _gpu_vjp(g, s, lam, dt)
    rng = np.random.default_rng(43)
    worst = 0.0
    for rep in range(3):
        delta = {f: rng.standard_normal(g.field_shape(f)) for f in FIELDS}
        I._periodic_face_copy(g, delta)
        _, jv, st = cso.jvp(g, s, delta, [dt])
        assert st == 0
        want = sum(float(np.sum(lam[f] * jv[f])) for f in FIELDS)
        scale = sum(float(np.sum(np.abs(lam[f] * jv[f]))) for f in FIELDS)
        got = sum(float(np.sum(lin[f] * delta[f])) for f in FIELDS)
        worst = max(worst, abs(got - want) / scale)
    for f in FIELDS:
        shape = list(g.field_shape(f))
        for _ in range(3):
            idx = tuple(int(rng.integers(0, m - (1 if (f, a) in (("bx", 2), ("by", 1), ("bz", 0)) else 0)))
                        for a, m in enumerate(shape))
            e = _unit(g, f, idx)
            _, jv, _ = cso.jvp(g, s, e, [dt])
            want = sum(float(np.sum(lam[q] * jv[q])) for q in FIELDS)
            scale = sum(float(np.sum(np.abs(lam[q] * jv[q]))) for q in FIELDS)
            worst = max(worst, abs(float(lin[f][idx]) - want) / scale)
    _say("recon %d: worst rel err against complex step %.2e" % (recon, worst))
    assert worst <= 1e-10


@pytest.mark.parametrize("admarch", [8, 16])
@pytest.mark.parametrize("recon", [I.RECON_PLMC, I.RECON_PLMP, I.RECON_PPMC, I.RECON_PPMP])
def test_adjoint_complex_step_multi_segment_grid(cso, recon, admarch, monkeypatch):
    """A 40 x 36 x 34 grid: rows longer than one block of the x-face kernel
    and several segments per column of the y and z marches (the segment
    boundaries, the face a segment computes beyond its top cell).  The size
    rule would pick 8-cell segments for the linear reconstructions' fused
    marches on a grid this small; the tile override (VLCT_TILES) runs both
    the 8- and the 16-cell variant (the one large grids use).
    <lam_in, delta> against the complex step of the oracle along random
    directions, within 1e-10."""
    _need_gpu()
    monkeypatch.setenv("VLCT_TILES", "admarch=%d" % admarch)
    g, s = _state((40, 36, 34), recon, 7)
    dt = ref.cfl_dt(g, s)
    lam = _random_cotangent(g, 3)
    lin = _gpu_vjp(g, s, lam, dt)
    rng = np.random.default_rng(5)
    worst = 0.0
    for _ in range(2):
        delta = {f: rng.standard_normal(g.field_shape(f)) for f in FIELDS}
        I._periodic_face_copy(g, delta)
        _, jv, st = cso.jvp(g, s, delta, [dt])
        assert st == 0
        want = sum(float(np.sum(lam[f] * jv[f])) for f in FIELDS)
        scale = sum(float(np.sum(np.abs(lam[f] * jv[f]))) for f in FIELDS)
        got = sum(float(np.sum(lin[f] * delta[f])) for f in FIELDS)
        worst = max(worst, abs(got - want) / scale)
    _say("recon %d, 40x36x34: worst rel err against complex step %.2e" % (recon, worst))
    assert worst <= 1e-10



@pytest.mark.parametrize("shape", [(16, 12, 1), (1, 9, 10), (12, 1, 11), (10, 2, 9)])
@pytest.mark.parametrize("recon", [I.RECON_PLMC, I.RECON_PPMC, I.RECON_PLMP, I.RECON_PPMP])
def test_adjoint_complex_step_thin_grids(cso, recon, shape):
    """Periodic grids one cell thick along each axis in turn, and two cells
    thick along y: a cell is then its own neighbour (or its neighbour's
    neighbour), so the reversal's accumulation into the stencil cells and the
    marches' and rows' hand-offs wrap onto the same cells.  <lam_in, delta>
    against the complex step of the oracle along random directions, within
    1e-10."""
    _need_gpu()
    from test_gpu_parity import _shaped_state
    g, s = _shaped_state(shape, recon, (0, 0, 0), 21)
    dt = ref.cfl_dt(g, s)
    lam = _random_cotangent(g, 22)
    lin = _gpu_vjp(g, s, lam, dt)
    rng = np.random.default_rng(23)
    worst = 0.0
    for _ in range(3):
        delta = {f: rng.standard_normal(g.field_shape(f)) for f in FIELDS}
        I._periodic_face_copy(g, delta)
        _, jv, st = cso.jvp(g, s, delta, [dt])
        assert st == 0
        want = sum(float(np.sum(lam[f] * jv[f])) for f in FIELDS)
        scale = sum(float(np.sum(np.abs(lam[f] * jv[f]))) for f in FIELDS)
        got = sum(float(np.sum(lin[f] * delta[f])) for f in FIELDS)
        worst = max(worst, abs(got - want) / scale)
    _say("recon %d, %s: worst rel err against complex step %.2e" % (recon, shape, worst))
    assert worst <= 1e-10
