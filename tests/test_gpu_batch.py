"""Batched ensembles on the GPU (vlct_step_batch): independent instances of
different sizes, gamma, boundaries and dt advanced together must each give
exactly what vlct_step gives for them alone (same kernels, same arithmetic),
and so match the oracle to the parity bar."""
import numpy as np
import pytest

from oracle import ref
from paper_2402_05240_amd import inputs as I
from parity_util import FIELDS, gpu_available, rel_l1, scales

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _say(msg):
    print(msg, flush=True)


def _instances(recon):
    out = [I.turbulence((22, 19, 17), recon=recon),
           I.blast((13, 12, 10), b0=1.0, recon=recon),
           I.turbulence((9, 31, 10), recon=recon, seed_v=7, seed_a=8),
           I.uniform((5, 7, 4), rho=1.1, v=(0.3, -0.2, 0.1), p=0.8, b=(0.5, 0.2, -0.3),
                     gamma=1.4, recon=recon, bc=(1, 0, 1)),
           I.linear_wave((24, 8, 8), "fast", recon=recon)[:2],
           I.turbulence((33, 20, 17), recon=recon, gamma=1.4)]
    return out


def _single(g, s0, dt, nsteps):
    from paper_2402_05240_amd.device import Stepper
    import torch
    st = Stepper(g).upload(s0)
    st.set_dt(dt)
    nexts = []
    for _ in range(nsteps):
        st.step()
        nexts.append(float(st.dt.item()))
    torch.cuda.synchronize()
    return st.download(), nexts, st.status_bits()


@pytest.mark.parametrize("recon,nsteps", [(2, 3), (3, 2)])
def test_batch_equals_single_instances(recon, nsteps):
    _need_gpu()
    from paper_2402_05240_amd.device import BatchStepper
    import torch
    inst = _instances(recon)
    grids = [g for g, _ in inst]
    dts = [ref.cfl_dt(g, s) for g, s in inst]
    _say("batch of %d instances, recon %d, %d steps" % (len(inst), recon, nsteps))
    bs = BatchStepper(grids).upload([s for _, s in inst])
    bs.set_dt(dts)
    nexts = []
    for _ in range(nsteps):
        bs.step()
        nexts.append(bs.dt.cpu().numpy().copy())
    torch.cuda.synchronize()
    outs = bs.download()
    status = bs.status_bits()
    for q, ((g, s0), dt) in enumerate(zip(inst, dts)):
        _say("single instance %d: %s" % (q, (g.nx, g.ny, g.nz)))
        ref_out, ref_nexts, ref_status = _single(g, s0, dt, nsteps)
        for f in FIELDS:
            assert np.array_equal(outs[q][f], ref_out[f]), (q, f)
        assert [float(n[q]) for n in nexts] == ref_nexts, q
        assert status[q] == ref_status, q


def test_batch_extreme_shapes_equal_single_instances():
    """Instances at the shape limits in one batch (a 4096-cell side, grids one
    cell thick along one or two axes, outflow and periodic, next to an
    ordinary grid): each equals its single-instance run bit for bit."""
    _need_gpu()
    from paper_2402_05240_amd.device import BatchStepper
    import torch
    from test_gpu_parity import _shaped_state
    inst = [_shaped_state((4096, 3, 2), 2, (0, 0, 0), 7), _shaped_state((1, 7, 5), 2, (0, 0, 0), 8),
            _shaped_state((6, 1, 1), 2, (1, 0, 0), 9), _shaped_state((11, 10, 9), 2, (0, 1, 0), 10)]
    dts = [ref.cfl_dt(g, s) for g, s in inst]
    _say("batch of %d extreme-shape instances" % len(inst))
    bs = BatchStepper([g for g, _ in inst]).upload([s for _, s in inst])
    bs.set_dt(dts)
    for _ in range(3):
        bs.step()
    torch.cuda.synchronize()
    outs = bs.download()
    status = bs.status_bits()
    for q, ((g, s0), dt) in enumerate(zip(inst, dts)):
        _say("single instance %d: %s" % (q, (g.nx, g.ny, g.nz)))
        ref_out, _, ref_status = _single(g, s0, dt, 3)
        for f in FIELDS:
            assert np.array_equal(outs[q][f], ref_out[f]), (q, f)
        assert status[q] == ref_status, q


def test_batch_instance_matches_oracle():
    _need_gpu()
    from paper_2402_05240_amd.device import BatchStepper
    import torch
    inst = [I.turbulence((20, 18, 15)), I.blast((16, 14, 12), b0=1.0, recon=2)]
    bs = BatchStepper([g for g, _ in inst]).upload([s for _, s in inst])
    dts = [ref.cfl_dt(g, s) for g, s in inst]
    bs.set_dt(dts)
    for _ in range(5):
        bs.step()
    torch.cuda.synchronize()
    outs = bs.download()
    for (g, s0), dt, out in zip(inst, dts, outs):
        orc, _, _ = ref.run(g, s0, 5, dt0=dt)
        r = rel_l1(out, orc, scales(g, s0))
        _say("rel L1 %s" % {f: "%.1e" % r[f] for f in FIELDS})
        for f in FIELDS:
            assert r[f] <= 1e-12, (f, r[f])


def test_batch_inplace_equals_out_of_place():
    _need_gpu()
    from paper_2402_05240_amd.device import BatchStepper
    import torch
    inst = _instances(2)[:3]
    dts = [ref.cfl_dt(g, s) for g, s in inst]
    res = []
    for inplace in (False, True):
        bs = BatchStepper([g for g, _ in inst], inplace=inplace).upload([s for _, s in inst])
        bs.set_dt(dts)
        for _ in range(2):
            bs.step()
        torch.cuda.synchronize()
        res.append(bs.download())
    for a, b in zip(*res):
        for f in FIELDS:
            assert np.array_equal(a[f], b[f]), f


def test_batch_steps_replayed_from_hip_graph():
    """Two batched steps captured into one graph (A -> B -> A) and replayed
    three times, with eager work and a synchronisation between replays; every
    replay equals eager stepping bit for bit."""
    _need_gpu()
    from paper_2402_05240_amd.device import BatchStepper
    import torch
    inst = _instances(2)[:4]
    grids = [g for g, _ in inst]
    dts = [ref.cfl_dt(g, s) for g, s in inst]
    eager = BatchStepper(grids).upload([s for _, s in inst])
    eager.set_dt(dts)
    graphed = BatchStepper(grids).upload([s for _, s in inst])
    graphed.set_dt(dts)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        graphed.step()
        graphed.step()
    torch.cuda.synchronize()
    for rep in range(3):
        _say("replay %d" % rep)
        graph.replay()
        eager.step()
        eager.step()
        torch.cuda.synchronize()
        a, b = graphed.download(), eager.download()
        for q in range(len(inst)):
            for f in FIELDS:
                assert np.array_equal(a[q][f], b[q][f]), (rep, q, f)
        assert torch.equal(graphed.dt, eager.dt)


def _run_plan(inst, dts, plan, nsteps=2):
    from paper_2402_05240_amd.device import BatchStepper
    import torch
    bs = BatchStepper([g for g, _ in inst], plan=plan).upload([s for _, s in inst])
    bs.set_dt(dts)
    nexts = []
    for _ in range(nsteps):
        bs.step()
        nexts.append(bs.dt.cpu().numpy().copy())
    torch.cuda.synchronize()
    return bs.download(), nexts


def test_batch_tile_plans_are_bit_identical():
    """Every per-instance tile plan (CT tiles 64x8, 32x16, 16x32; march
    segments 16, 32, 8) gives exactly the default plan's results: the tiles
    only regroup the same per-cell and per-face arithmetic."""
    _need_gpu()
    inst = _instances(2)
    dts = [ref.cfl_dt(g, s) for g, s in inst]
    base, base_dt = _run_plan(inst, dts, None)
    rng = np.random.default_rng(3)
    plans = [[0x11] * len(inst), [0x22] * len(inst), [0x02] * len(inst),
             [int(rng.integers(0, 3)) | (int(rng.integers(0, 3)) << 4) for _ in inst]]
    for plan in plans:
        _say("plan %s" % [hex(p) for p in plan])
        outs, nexts = _run_plan(inst, dts, plan)
        for q in range(len(inst)):
            for f in FIELDS:
                assert np.array_equal(outs[q][f], base[q][f]), (plan, q, f)
        for a, b in zip(nexts, base_dt):
            assert np.array_equal(a, b)


def test_batch_autotuner_plan_is_valid_and_exact():
    _need_gpu()
    from paper_2402_05240_amd.device import BatchStepper
    import torch
    ens = I.ensemble(12, seed=7, nmin=16, nmax=64)
    inst = [(g, s) for g, s, _ in ens]
    dts = [ref.cfl_dt(g, s) for g, s in inst]
    tuner = BatchStepper([g for g, _ in inst]).upload([s for _, s in inst])
    tuner.set_dt(dts)
    plan = tuner.tune(reps=2)
    torch.cuda.synchronize()
    _say("tuned plan %s" % [hex(p) for p in plan])
    assert len(plan) == len(inst)
    assert all((p & 15) < 3 and (p >> 4) < 3 for p in plan)
    # the tuner leaves the input states untouched
    for d, (g, s) in zip(tuner.download(), inst):
        for f in FIELDS:
            assert np.array_equal(d[f], s[f])
    base, _ = _run_plan(inst, dts, None, nsteps=1)
    tuned, _ = _run_plan(inst, dts, plan, nsteps=1)
    for q in range(len(inst)):
        for f in FIELDS:
            assert np.array_equal(tuned[q][f], base[q][f]), (q, f)


def test_batch_until_each_instance_to_its_own_end_time():
    """vlct_step_batch_until: instances with different periods each run to
    their own end time (the last step clipped onto it) and then drop out;
    every instance ends bit for bit where vlct_step gets it with the same
    clip, and the times land on the end times."""
    _need_gpu()
    import torch
    from paper_2402_05240_amd.device import BatchStepper, Stepper
    ens = I.ensemble(5, seed=11, nmin=12, nmax=24)
    grids = [g for g, _, _ in ens]
    ends = [0.25 * T * (1 + q) / 5 for q, (_, _, T) in enumerate(ens)]
    _say("ensemble of %d, end times %s" % (len(ens), ["%.3g" % x for x in ends]))
    bs = BatchStepper(grids, inplace=True).upload([s for _, s, _ in ens])
    bs.compute_dt()
    nb = bs.run_until(ends, check_every=4)
    got = bs.download()
    t_b = bs.t.cpu().numpy()
    counts = []
    for q, ((g, s, _), tend) in enumerate(zip(ens, ends)):
        st = Stepper(g, inplace=True).upload(s)
        st.compute_dt()
        t = torch.zeros(1, dtype=torch.float64, device="cuda")
        te = torch.tensor([tend], dtype=torch.float64, device="cuda")
        n = 0
        while float(t.item()) < tend:
            dte = torch.minimum(st.dt, te - t)
            st.dt.copy_(dte)
            st.step()
            t += dte
            n += 1
        counts.append(n)
        ref_state = st.download()
        assert float(t.item()) == t_b[q], q
        for f in FIELDS:
            assert np.array_equal(got[q][f], ref_state[f]), (q, f)
    _say("steps per instance %s, batched steps %d" % (counts, nb))
    assert len(set(counts)) > 1 and nb >= max(counts)
    assert np.allclose(t_b, ends, rtol=1e-14, atol=0)
