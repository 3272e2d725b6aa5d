"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/vlct.h declares, argument validation returns
the documented codes before anything is launched, and the full-size sampling
used by the GPU parity tests reproduces the oracle exactly."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import ref
from paper_2402_05240_amd import inputs as I
from paper_2402_05240_amd import vlct
from parity_util import ROOT, WINDOW_HALF, cell_values, window


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "vlct.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vlct_\w+)\s*\(", src)))


def _lib():
    if not os.path.exists(vlct.LIB_PATH):
        pytest.skip("libvlct.so not built")
    return vlct.load()


def test_library_exports_every_declared_function():
    lib = _lib()
    decl = _declared_functions()
    assert set(decl) == set(vlct.EXPORTED)
    for name in decl:
        assert hasattr(lib, name), name
    assert vlct.vlct_abi_version() == 100


# spacing of fake device addresses in the validation tests: more than any
# field of the test grids, so fake arrays never overlap unless a test says so
SPACING = 1 << 20


def _grid(**kw):
    base = dict(nx=8, ny=8, nz=8, dx=0.1, dy=0.1, dz=0.1, gamma=5 / 3, cfl=0.4, recon=2, bc=(0, 0, 0))
    base.update(kw)
    return vlct.make_grid(I.Grid(**base))


@pytest.mark.parametrize("bad", [dict(nx=0), dict(ny=-3), dict(nz=5000), dict(dx=0.0), dict(dy=-1.0),
                                 dict(dz=float("nan")), dict(gamma=1.0), dict(cfl=0.0), dict(cfl=0.6),
                                 dict(recon=0), dict(recon=6), dict(bc=(0, 2, 0))])
def test_invalid_grid_rejected(bad):
    _lib()
    g = _grid(**bad)
    assert vlct.vlct_workspace_bytes(g) == 0
    fake = vlct.make_state([16] * 8)
    rc = vlct.vlct_step(g, fake, fake, 16, 16, 0, 16, 1 << 40, 0)
    assert rc == vlct.VLCT_EINVAL
    assert vlct.vlct_cfl_dt(g, fake, 16, 16, 1 << 40, 0) == vlct.VLCT_EINVAL


def test_workspace_and_pointer_validation():
    _lib()
    g = _grid()
    need = vlct.vlct_workspace_bytes(g)
    assert need > 8 * 8 ** 3 * 8
    fake = vlct.make_state([SPACING * (f + 1) for f in range(8)])
    # missing / short workspace
    assert vlct.vlct_step(g, fake, fake, 64, 0, 0, 0, need, 0) == vlct.VLCT_EWORKSPACE
    assert vlct.vlct_step(g, fake, fake, 64, 0, 0, 128, need - 1, 0) == vlct.VLCT_EWORKSPACE
    assert vlct.vlct_cfl_dt(g, fake, 64, 128, need - 1, 0) == vlct.VLCT_EWORKSPACE
    # NULL field, NULL dt
    holey = vlct.make_state([SPACING * (f + 1) for f in range(7)] + [0])
    assert vlct.vlct_step(g, holey, fake, 64, 0, 0, 128, need, 0) == vlct.VLCT_EINVAL
    assert vlct.vlct_step(g, fake, fake, 0, 0, 0, 128, need, 0) == vlct.VLCT_EINVAL
    # partial aliasing of out and in: shared base pointers
    other = vlct.make_state([SPACING * (f + 1) for f in range(7)] + [10 ** 9])
    part = vlct.make_state([10 ** 9 + SPACING * f for f in range(7)] + [SPACING])
    assert vlct.vlct_step(g, fake, part, 64, 0, 0, 128, need, 0) == vlct.VLCT_EINVAL
    assert vlct.vlct_step(g, fake, other, 64, 0, 0, 128, need, 0) == vlct.VLCT_EINVAL


def test_overlapping_address_ranges_rejected():
    """Output arrays must not overlap an input array or each other as address
    ranges, even when no two base pointers are equal (an 8^3 cell field is
    4096 bytes, a face field 4608)."""
    _lib()
    g = _grid()
    need = vlct.vlct_workspace_bytes(g)
    fin = vlct.make_state([SPACING * (f + 1) for f in range(8)])
    ok_out = vlct.make_state([10 ** 9 + SPACING * f for f in range(8)])
    # a valid out-of-place call reaches the workspace check
    assert vlct.vlct_step(g, fin, ok_out, 64, 0, 0, 0, need, 0) == vlct.VLCT_EWORKSPACE
    # out.E starts 8 bytes into in.E; out.rho ends one double into in.rho
    shifted = vlct.make_state([10 ** 9 + SPACING * f for f in range(4)] + [SPACING * 5 + 8]
                              + [10 ** 9 + SPACING * f for f in range(5, 8)])
    assert vlct.vlct_step(g, fin, shifted, 64, 0, 0, 128, need, 0) == vlct.VLCT_EINVAL
    tail = vlct.make_state([SPACING * 1 - 4096 + 8] + [10 ** 9 + SPACING * f for f in range(1, 8)])
    assert vlct.vlct_step(g, fin, tail, 64, 0, 0, 128, need, 0) == vlct.VLCT_EINVAL
    # two outputs overlapping each other: bx (4608 bytes) runs into by
    twin = vlct.make_state([10 ** 9 + SPACING * f for f in range(5)]
                           + [10 ** 9 + SPACING * 5, 10 ** 9 + SPACING * 5 + 4096,
                              10 ** 9 + SPACING * 7])
    assert vlct.vlct_step(g, fin, twin, 64, 0, 0, 128, need, 0) == vlct.VLCT_EINVAL
    # just touching ranges are fine
    touch = vlct.make_state([SPACING * 1 + 4096] + [10 ** 9 + SPACING * f for f in range(1, 8)])
    assert vlct.vlct_step(g, fin, touch, 64, 0, 0, 0, need, 0) == vlct.VLCT_EWORKSPACE


def test_noalloc_validation():
    """vlct_step_noalloc checks its arguments and the scratch size on the host,
    before it looks up the scratch or launches anything."""
    _lib()
    fake = vlct.make_state([SPACING * (f + 1) for f in range(8)])
    assert vlct.vlct_step_noalloc(_grid(nx=0), fake, fake, 64, 0, 0, 0) == vlct.VLCT_EINVAL
    assert vlct.vlct_step_noalloc(_grid(), fake, fake, 0, 0, 0, 0) == vlct.VLCT_EINVAL
    holey = vlct.make_state([SPACING * (f + 1) for f in range(7)] + [0])
    assert vlct.vlct_step_noalloc(_grid(), holey, fake, 64, 0, 0, 0) == vlct.VLCT_EINVAL
    big = _grid(nx=96, ny=96, nz=96)
    assert vlct.vlct_workspace_bytes(big) > vlct.VLCT_NOALLOC_SCRATCH_BYTES
    assert vlct.vlct_step_noalloc(big, fake, fake, 64, 0, 0, 0) == vlct.VLCT_ESCRATCH
    fits = _grid(nx=48, ny=48, nz=48)
    assert vlct.vlct_workspace_bytes(fits) <= vlct.VLCT_NOALLOC_SCRATCH_BYTES


def test_batch_validation():
    """vlct_step_batch rejects bad calls on the host, before any launch."""
    _lib()
    g1, g2 = _grid(), _grid(nx=12, ny=5, nz=7, bc=(1, 0, 1))
    assert vlct.vlct_batch_workspace_bytes([]) == 0
    one = vlct.vlct_batch_workspace_bytes([g1])
    two = vlct.vlct_batch_workspace_bytes([g1, g2])
    assert two > one > vlct.vlct_workspace_bytes(g1)
    assert two >= vlct.vlct_workspace_bytes(g1) + vlct.vlct_workspace_bytes(g2)
    assert vlct.vlct_batch_workspace_bytes([g1, _grid(nx=0)]) == 0

    def st(base):
        return vlct.make_state([base + 4096 * f for f in range(8)])
    a, b, c, d = st(1 << 20), st(2 << 20), st(3 << 20), st(4 << 20)
    ws = 1 << 30
    # empty batch, NULL dt, invalid member
    assert vlct.vlct_step_batch([], [], [], 64, 0, 0, ws, two, 0) == vlct.VLCT_EINVAL
    assert vlct.vlct_step_batch([g1, g2], [a, b], [c, d], 0, 0, 0, ws, two, 0) == vlct.VLCT_EINVAL
    assert vlct.vlct_step_batch([g1, _grid(dx=0.0)], [a, b], [c, d], 64, 0, 0, ws, two,
                                0) == vlct.VLCT_EINVAL
    # mixed reconstructions
    assert vlct.vlct_step_batch([g1, _grid(recon=3)], [a, b], [c, d], 64, 0, 0, ws, two,
                                0) == vlct.VLCT_EUNSUPPORTED
    # an output shared by two instances, an input that is another instance's output
    assert vlct.vlct_step_batch([g1, g2], [a, b], [c, c], 64, 0, 0, ws, two, 0) == vlct.VLCT_EINVAL
    assert vlct.vlct_step_batch([g1, g2], [a, c], [c, d], 64, 0, 0, ws, two, 0) == vlct.VLCT_EINVAL
    # workspace missing or short
    assert vlct.vlct_step_batch([g1, g2], [a, b], [c, d], 64, 0, 0, 0, two,
                                0) == vlct.VLCT_EWORKSPACE
    assert vlct.vlct_step_batch([g1, g2], [a, b], [c, d], 64, 0, 0, ws, two - 1,
                                0) == vlct.VLCT_EWORKSPACE


def test_batch_plan_and_tune_validation():
    """Unknown tile variants and in-place tuning are rejected on the host."""
    _lib()
    g1, g2 = _grid(), _grid(nx=12, ny=5, nz=7)
    two = vlct.vlct_batch_workspace_bytes([g1, g2])

    def st(base):
        return vlct.make_state([base + 4096 * f for f in range(8)])
    a, b, c, d = st(1 << 20), st(2 << 20), st(3 << 20), st(4 << 20)
    ws = 1 << 30
    for bad in ([3, 0], [0, 0x30], [0, 0xF3]):
        assert vlct.vlct_step_batch_plan([g1, g2], [a, b], [c, d], 64, 0, 0, bad, ws, two,
                                         0) == vlct.VLCT_EINVAL
    # tuning steps write `out`: an in-place instance is refused
    rc, _ = vlct.vlct_batch_tune([g1, g2], [a, b], [a, d], 64, ws, two, 0)
    assert rc == vlct.VLCT_EINVAL
    rc, _ = vlct.vlct_batch_tune([g1, g2], [a, b], [c, d], 64, ws, two, 0, reps=0)
    assert rc == vlct.VLCT_EINVAL
    rc, _ = vlct.vlct_batch_tune([g1, g2], [a, b], [c, d], 64, ws, two - 1, 0)
    assert rc == vlct.VLCT_EWORKSPACE


def test_adjoint_validation():
    """vlct_step_adjoint rejects bad calls on the host, before any launch."""
    _lib()
    g = _grid()
    need = vlct.vlct_adjoint_workspace_bytes(g)
    assert need > vlct.vlct_workspace_bytes(g)
    assert vlct.vlct_adjoint_workspace_bytes(_grid(nx=0)) == 0

    def st(base):
        return vlct.make_state([base + 8192 * f for f in range(8)])
    a, b, c = st(1 << 20), st(2 << 20), st(3 << 20)
    ws = 1 << 30
    assert vlct.vlct_step_adjoint(g, a, b, c, 0, ws, need, 0) == vlct.VLCT_EINVAL
    assert vlct.vlct_step_adjoint(_grid(dx=0.0), a, b, c, 64, ws, need, 0) == vlct.VLCT_EINVAL
    # outflow boundaries are not differentiated
    assert vlct.vlct_step_adjoint(_grid(bc=(0, 1, 0)), a, b, c, 64, ws, need,
                                  0) == vlct.VLCT_EUNSUPPORTED
    # lam_in overlapping the state, lam_out or itself
    assert vlct.vlct_step_adjoint(g, a, b, a, 64, ws, need, 0) == vlct.VLCT_EINVAL
    assert vlct.vlct_step_adjoint(g, a, b, st((2 << 20) + 8), 64, ws, need, 0) == vlct.VLCT_EINVAL
    same = vlct.make_state([3 << 20] * 8)
    assert vlct.vlct_step_adjoint(g, a, b, same, 64, ws, need, 0) == vlct.VLCT_EINVAL
    # workspace missing or short
    assert vlct.vlct_step_adjoint(g, a, b, c, 64, 0, need, 0) == vlct.VLCT_EWORKSPACE
    assert vlct.vlct_step_adjoint(g, a, b, c, 64, ws, need - 1, 0) == vlct.VLCT_EWORKSPACE


def test_taped_validation():
    """vlct_step_taped / vlct_step_adjoint_taped reject bad calls on the host."""
    _lib()
    g = _grid()
    tb = vlct.vlct_tape_bytes(g)
    assert tb > 0 and vlct.vlct_tape_bytes(_grid(nx=0)) == 0
    wt = vlct.vlct_adjoint_taped_workspace_bytes(g)
    assert 0 < wt < vlct.vlct_adjoint_workspace_bytes(g)
    ws_step = vlct.vlct_workspace_bytes(g)

    def st(base):
        return vlct.make_state([base + 8192 * f for f in range(8)])
    a, b, c = st(1 << 20), st(2 << 20), st(3 << 20)
    big = 1 << 30
    assert vlct.vlct_step_taped(g, a, b, 64, 0, 0, big, ws_step, big, tb - 1, 0) == vlct.VLCT_EWORKSPACE
    assert vlct.vlct_step_taped(g, a, b, 64, 0, 0, big, ws_step, 0, tb, 0) == vlct.VLCT_EWORKSPACE
    assert vlct.vlct_step_taped(g, a, b, 0, 0, 0, big, ws_step, big, tb, 0) == vlct.VLCT_EINVAL
    assert vlct.vlct_step_adjoint_taped(g, a, b, c, 64, big, tb - 1, big, wt,
                                        0) == vlct.VLCT_EWORKSPACE
    assert vlct.vlct_step_adjoint_taped(g, a, b, c, 64, big, tb, big, wt - 1,
                                        0) == vlct.VLCT_EWORKSPACE
    assert vlct.vlct_step_adjoint_taped(_grid(bc=(1, 0, 0)), a, b, c, 64, big, tb, big, wt,
                                        0) == vlct.VLCT_EUNSUPPORTED
    assert vlct.vlct_step_adjoint_taped(g, a, b, a, 64, big, tb, big, wt, 0) == vlct.VLCT_EINVAL


def test_strerror_covers_codes():
    _lib()
    for c in range(6):
        assert vlct.vlct_strerror(c)
        assert "unknown" not in vlct.vlct_strerror(c)
    assert "unknown" in vlct.vlct_strerror(99)


def test_missing_library_fails_loudly(tmp_path):
    saved = vlct._lib
    try:
        vlct._lib = None
        with pytest.raises(RuntimeError):
            vlct.load(str(tmp_path / "nope.so"))
    finally:
        vlct._lib = saved


@pytest.mark.parametrize("maker", ["turb_plmc", "turb_ppmc", "blast"])
def test_window_sampling_reproduces_full_oracle(maker):
    """A cell of a one-step result depends only on cells within 4 of it, so
    the oracle run on a window around a sampled cell equals the full run
    there; the full-size GPU parity tests rely on this."""
    if maker == "turb_plmc":
        g, s = I.turbulence((16, 16, 16))
    elif maker == "turb_ppmc":
        g, s = I.turbulence((16, 16, 16), recon=3)
    else:
        g, s = I.blast((16, 16, 16), b0=1.0)
    dt = ref.cfl_dt(g, s)
    full, _, _ = ref.step(g, s, dt, nthreads=2)
    rng = np.random.default_rng(3)
    cells = [(0, 15, 7), (15, 0, 0)] + [tuple(int(x) for x in rng.integers(0, 16, 3)) for _ in range(3)]
    for c in cells:
        wg, ws, cw = window(g, s, c, 4)
        wout, _, _ = ref.step(wg, ws, dt, nthreads=1)
        assert np.array_equal(cell_values(wg, wout, cw), cell_values(g, full, c))
    assert WINDOW_HALF >= 4
