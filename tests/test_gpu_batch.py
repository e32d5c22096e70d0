"""GPU parity of the batched instances (fused step over a work list of tiles
of many grids) against the FP64 oracle, instance by instance."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) /
                 np.linalg.norm(np.asarray(b).ravel()))


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1906_06327_amd as P
    P.lib()
    return P


def mixed(prec, mode=0):
    # nx = 129 takes 16 lines per x-sweep block (nx * L > 2048): the batch then
    # stages 16 points per x-sweep thread instead of 8
    shapes = [(100, 77), (64, 64), (130, 47), (33, 200), (128, 128), (129, 40)]
    out = []
    for t, (nx, ny) in enumerate(shapes):
        out.append(dict(dim=2, nx=nx, ny=ny, nz=1, hx=0.1 + 0.01 * t, hy=0.09 + 0.005 * t, hz=0.1,
                        gamma=1.0, nu=1.0 + 0.05 * t, lam=1.0, g=30.0 + 25.0 * t,
                        omega=0.3 + 0.1 * t, dt=1e-3 * (1 + t % 2), mode=mode, precision=prec))
    return out


@pytest.mark.parametrize("plan", [1, 2])
@pytest.mark.parametrize("prec,mode", [(0, 0), (0, 1), (1, 0)])
def test_batch_step_matches_oracle_per_instance(P, prec, mode, plan):
    print(f"[gpu-batch] step prec={prec} mode={mode} plan={plan}", flush=True)
    cfgs = mixed(prec, mode)
    b = P.Batch(cfgs)
    b.set_plan(plan)
    refs = []
    for k, c in enumerate(cfgs):
        ph = W.phase_field(30 + k, c["ny"], c["nx"])
        b.init_state(k, 1, ph, 1.0)
        op = O.make_params(**c)
        refs.append((op, O.init_state(op, 1, ph, 1.0)))
    b.step(77)
    tol = 1e-10 if prec == 0 else 1e-5
    obs = b.observables()
    for k, (op, r0) in enumerate(refs):
        ref = O.step(op, r0, 77)
        got = b.get_state(k).astype(np.complex128)
        assert rel(got, ref) <= tol, k
        oo = O.observables(op, ref)
        for key in ("norm", "mu", "energy", "rms_x"):
            assert abs(obs[k][key] - oo[key]) <= tol * max(1.0, abs(oo[key])), (k, key)
    b.close()


@pytest.mark.parametrize("plan", [0, 1, 2])
def test_batch_run_drops_converged_instances(P, plan):
    """Instances converge at different steps; each stops exactly there: its
    state equals the oracle's after that many steps (either plan, or the
    one the autotuner picks)."""
    print(f"[gpu-batch] run to convergence plan={plan}", flush=True)
    cfgs = []
    for t in range(4):
        cfgs.append(dict(dim=2, nx=48 + 8 * t, ny=44 + 4 * t, nz=1, hx=0.25, hy=0.25, hz=0.1,
                         gamma=1.0, nu=1.1, lam=1.0, g=5.0 + 20.0 * t, omega=0.2 + 0.1 * t,
                         dt=0.02, mode=0, precision=0))
    b = P.Batch(cfgs)
    if plan:
        b.set_plan(plan)
    for k, c in enumerate(cfgs):
        b.init_state(k, 0, W.phase_field(50 + k, c["ny"], c["nx"]), 1.0)
    steps = b.run(max_steps=20000, check_every=50, tol=1e-9)
    assert b.info()["plan"] in (1, 2)
    assert all(s > 0 for s in steps), steps
    assert len(set(steps)) > 1, steps  # they do not all stop together
    for k, c in enumerate(cfgs):
        op = O.make_params(**c)
        ref = O.step(op, O.init_state(op, 0, W.phase_field(50 + k, c["ny"], c["nx"]), 1.0), steps[k])
        assert rel(b.get_state(k), ref) <= 1e-10, k
    b.close()


@pytest.mark.parametrize("plan", [1, 2])
def test_batch_workload_sampled(P, plan):
    """The 64-instance workload at full size: a few steps, sampled instances
    against the oracle."""
    print(f"[gpu-batch] 64-instance workload plan={plan}", flush=True)
    cfgs = W.batch_instances()
    b = P.Batch(cfgs)
    b.set_plan(plan)
    for k, c in enumerate(cfgs):
        b.init_state(k, 1, W.phase_field(c["seed"], c["ny"], c["nx"]), 1.0)
    b.step(10)
    for k in (0, 17, 40, 63):
        c = cfgs[k]
        op = O.make_params(**c)
        ref = O.step(op, O.init_state(op, 1, W.phase_field(c["seed"], c["ny"], c["nx"]), 1.0), 10)
        assert rel(b.get_state(k), ref) <= 1e-10, k
    b.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_set_state_device_and_vortex_count(P, prec):
    """A state written into an instance's buffer gets zero walls and unit
    norm as the oracle's; the per-instance vortex count equals the oracle's."""
    import torch
    print(f"[gpu-batch] set_state_device prec={prec}", flush=True)
    cfgs = mixed(prec)[:3]
    b = P.Batch(cfgs)
    rng = np.random.default_rng(60 + prec)
    for k, c in enumerate(cfgs):
        ny, nx = c["ny"], c["nx"]
        y, x = np.mgrid[0:ny, 0:nx]
        z = (x - 0.37 * nx) + 1j * (y - 0.55 * ny)
        z2 = (x - 0.7 * nx) - 1j * (y - 0.3 * ny)
        f = z * z2 * np.exp(-((x - nx / 2) ** 2 + (y - ny / 2) ** 2) / (0.1 * nx * ny))
        f = f + 0.01 * (rng.standard_normal(f.shape) + 1j * rng.standard_normal(f.shape))
        b.psi[k].copy_(torch.tensor(f.astype(np.complex128 if prec == 0 else np.complex64)))
        b.set_state_device(k)
        op = O.make_params(**c)
        ref = np.asarray(f.astype(np.complex128 if prec == 0 else np.complex64), dtype=np.complex128)
        ref[0, :] = 0
        ref[:, 0] = 0
        ref = O.normalize(op, ref)
        got = b.get_state(k).astype(np.complex128)
        assert np.all(got[0, :] == 0) and np.all(got[:, 0] == 0)
        assert rel(got, ref) <= (1e-13 if prec == 0 else 1e-6), k
        assert b.vortex_count(k) == O.vortex_count(op, got), k
    b.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_groups_give_the_same_bits(P, prec, monkeypatch):
    """The sweep plan runs its instances group by group (groups sized for the
    Infinity Cache, SSCN_BATCH_GROUP_MB).  Instances are independent, so any
    grouping gives the same bits: one group per instance against one group
    for all, over direct steps, graph-replayed steps and a convergence run
    with drop-out, and each against the oracle."""
    print(f"[gpu-batch] groups prec={prec}", flush=True)
    cfgs = mixed(prec, 0)
    res = {}
    for mb in ("0", "1"):
        monkeypatch.setenv("SSCN_BATCH_GROUP_MB", mb)
        b = P.Batch(cfgs)
        b.set_plan(1)
        for k, c in enumerate(cfgs):
            b.init_state(k, 1, W.phase_field(40 + k, c["ny"], c["nx"]), 1.0)
        b.step(1)
        b.step(37)
        st = b.run(3000, check_every=100, tol=1e-5)
        res[mb] = ([b.get_state(k) for k in range(len(cfgs))], list(st), b.observables())
        b.close()
    for k in range(len(cfgs)):
        assert np.array_equal(res["0"][0][k], res["1"][0][k]), k
    assert res["0"][1] == res["1"][1]
    # and the grouped states match the oracle after the direct and replayed steps
    monkeypatch.setenv("SSCN_BATCH_GROUP_MB", "1")
    bb = P.Batch(cfgs)
    bb.set_plan(1)
    for k, c in enumerate(cfgs):
        bb.init_state(k, 1, W.phase_field(40 + k, c["ny"], c["nx"]), 1.0)
    bb.step(1)
    bb.step(37)
    tol = 1e-10 if prec == 0 else 1e-5
    for k, c in enumerate(cfgs):
        op = O.make_params(**c)
        ref = O.step(op, O.init_state(op, 1, W.phase_field(40 + k, c["ny"], c["nx"]), 1.0), 38)
        assert rel(bb.get_state(k).astype(np.complex128), ref) <= tol, k
    bb.close()


def x_option_runs(P, cfgs, monkeypatch, seed0):
    """States, convergence steps and observables of the same stepping under
    each x-sweep lines-per-block option (SSCN_BATCH_XLINES), and the
    autotuner's times with neither forced."""
    res = {}
    for opt in ("0", "1"):
        monkeypatch.setenv("SSCN_BATCH_XLINES", opt)
        b = P.Batch(cfgs)
        b.set_plan(1)
        for k, c in enumerate(cfgs):
            b.init_state(k, 1, W.phase_field(seed0 + k, c["ny"], c["nx"]), 1.0)
        b.step(1)
        b.step(37)
        st = b.run(3000, check_every=100, tol=1e-5)
        info = b.info()
        assert info["x_lines_option"] == int(opt) and info["x_lines_tune_ms"] == [0.0, 0.0]
        res[opt] = ([b.get_state(k) for k in range(len(cfgs))], list(st), b.observables())
        b.close()
    monkeypatch.delenv("SSCN_BATCH_XLINES")
    b = P.Batch(cfgs)
    b.set_plan(1)
    for k, c in enumerate(cfgs):
        b.init_state(k, 1, W.phase_field(seed0 + k, c["ny"], c["nx"]), 1.0)
    b.step(1)
    tune = b.info()["x_lines_tune_ms"]
    b.close()
    return res, tune


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_x_options_give_the_same_bits(P, prec, monkeypatch):
    """The batched x-sweep's two lines-per-block options (the most lines a
    block can stage, or that number halved until the block's LDS is at most
    40 KiB) only regroup whole lines into blocks, so they give the same bits,
    over direct steps, graph-replayed steps and a convergence run with
    drop-out, in 2D and in 3D (where the x-sweep works in place).  With
    neither forced, the autotuner times both where they differ (complex128:
    W = 13 puts the 16-line blocks of nx = 100, 128, 129 above 40 KiB) and
    neither where they coincide (complex64: W = 6, every block below)."""
    print(f"[gpu-batch] x options prec={prec}", flush=True)
    cfgs = mixed(prec, 0)
    res, tune = x_option_runs(P, cfgs, monkeypatch, 60)
    for k in range(len(cfgs)):
        assert np.array_equal(res["0"][0][k], res["1"][0][k]), k
    assert res["0"][1] == res["1"][1]
    assert res["0"][2] == res["1"][2]
    if prec == 0:
        assert tune[0] > 0 and tune[1] > 0, tune
    else:
        assert tune == [0.0, 0.0], tune
    if prec == 0:
        c3 = [dict(c, nx=128 + 8 * t, ny=20 + 4 * t) for t, c in enumerate(mixed3d(0, 0)[:2])]
        res3, tune3 = x_option_runs(P, c3, monkeypatch, 70)
        for k in range(len(c3)):
            assert np.array_equal(res3["0"][0][k], res3["1"][0][k]), k
        assert res3["0"][1] == res3["1"][1]
        assert tune3[0] > 0 and tune3[1] > 0, tune3


def mixed3d(prec, mode=0):
    shapes = [(24, 20, 12), (32, 16, 10), (20, 28, 14)]
    out = []
    for t, (nx, ny, nz) in enumerate(shapes):
        out.append(dict(dim=3, nx=nx, ny=ny, nz=nz, hx=0.3 + 0.02 * t, hy=0.28 + 0.01 * t, hz=0.35 - 0.03 * t,
                        gamma=1.0, nu=1.0 + 0.05 * t, lam=2.0 + t, g=20.0 + 15.0 * t,
                        omega=0.4 + 0.1 * t, dt=1e-3 * (1 + t % 2), mode=mode, precision=prec))
    return out


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_3d_rescale_summed_per_instance(P, prec):
    """An instance with more than 256 norm partials (96 x 88 x 10: 264 z
    tiles) makes the batch sum each instance's partials once per step before
    the x-sweep (k_batch_scale) instead of in every x-sweep block; the steps
    and the observables still follow the oracle instance by instance."""
    print(f"[gpu-batch] 3D per-instance rescale sum prec={prec}", flush=True)
    big = dict(mixed3d(prec)[0], nx=96, ny=88, nz=10, hx=0.25, hy=0.25, hz=0.3)
    cfgs = mixed3d(prec)[:2] + [big]
    b = P.Batch(cfgs)
    refs = []
    for k, c in enumerate(cfgs):
        ph = W.phase_field(80 + k, c["ny"], c["nx"])
        b.init_state(k, 1, ph, 1.0)
        op = O.make_params(**c)
        refs.append((op, O.init_state(op, 1, ph, 1.0)))
    b.step(1)
    b.step(30)
    tol = 1e-10 if prec == 0 else 1e-5
    obs = b.observables()
    for k, (op, r0) in enumerate(refs):
        ref = O.step(op, r0, 31)
        assert rel(b.get_state(k).astype(np.complex128), ref) <= tol, k
        oo = O.observables(op, ref)
        for key in ("norm", "mu", "energy"):
            assert abs(obs[k][key] - oo[key]) <= tol * max(1.0, abs(oo[key])), (k, key)
    b.close()


@pytest.mark.parametrize("prec,mode", [(0, 0), (0, 1), (1, 0)])
def test_batch_3d_matches_oracle_per_instance(P, prec, mode):
    """A batch of 3D instances of different shapes and parameters (x-, y-
    and z-sweeps over work lists of every instance), stepped directly and
    from graphs, against the oracle instance by instance; then a convergence
    run with drop-out and the z = 0 plane's vortex count."""
    print(f"[gpu-batch] 3D prec={prec} mode={mode}", flush=True)
    cfgs = mixed3d(prec, mode)
    b = P.Batch(cfgs)
    assert b.info()["plan"] == 1
    refs = []
    for k, c in enumerate(cfgs):
        ph = W.phase_field(50 + k, c["ny"], c["nx"])
        b.init_state(k, 1, ph, 1.0)
        op = O.make_params(**c)
        r0 = O.init_state(op, 1, ph, 1.0)
        assert rel(b.get_state(k), r0) <= (1e-14 if prec == 0 else 1e-6), k
        refs.append((op, r0))
    b.step(1)
    b.step(40)
    tol = 1e-10 if prec == 0 else 1e-5
    obs = b.observables()
    for k, (op, r0) in enumerate(refs):
        ref = O.step(op, r0, 41)
        got = b.get_state(k).astype(np.complex128)
        assert rel(got, ref) <= tol, k
        oo = O.observables(op, ref)
        for key in ("norm", "mu", "energy", "rms_z"):
            assert abs(obs[k][key] - oo[key]) <= tol * max(1.0, abs(oo[key])), (k, key)
    prof = b.profile_step(3)
    assert prof["z"] > 0 and prof["x"] > 0 and prof["y"] > 0
    if mode == 0:
        st = b.run(20000, check_every=100, tol=1e-4)
        assert all(v > 0 for v in st), st
        for k, c in enumerate(cfgs):
            op = O.make_params(**c)
            assert b.vortex_count(k) == O.vortex_count(op, b.get_state(k).astype(np.complex128))
    b.close()
