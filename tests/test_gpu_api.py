"""GPU tests of the stepping and robustness contracts of the C ABI: graph
replay for any step count, prepared steps, bitwise restarts in every plan,
non-finite states reported as SSCN_ENONFINITE, the batched convergence
criterion (vortex count included) against the single-instance one, and the
per-kernel profile of the batched step."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1906_06327_amd as P
    P.lib()
    return P


def announce(msg):
    print(f"[gpu-api] {msg}", flush=True)


def small(nx=70, ny=54, prec=0, mode=0, **kw):
    c = dict(dim=2, nx=nx, ny=ny, nz=1, hx=0.12, hy=0.11, hz=0.1, gamma=1.0, nu=1.1, lam=1.0, g=60.0,
             omega=0.5, dt=1e-3, mode=mode, precision=prec)
    c.update(kw)
    return c


@pytest.mark.parametrize("plan", [1, 2])
@pytest.mark.parametrize("prec", [0, 1])
def test_graph_steps_equal_single_steps(P, plan, prec):
    """A call of n steps (graphs of min(n, 64) steps and a remainder) leaves
    the same bits as n calls of one step (direct launches, each ending with
    its own rescale), for step counts below, at and above the graph size."""
    announce(f"graph vs single steps plan={plan} prec={prec}")
    cfg = small(prec=prec)
    ph = W.phase_field(3, cfg["ny"], cfg["nx"])
    for n in (2, 5, 64, 67, 129):
        a = P.Solver(W.solver_params(cfg))
        a.set_plan(plan)
        a.init_state(1, ph, 1.0)
        a.step(n)
        b = P.Solver(W.solver_params(cfg))
        b.set_plan(plan)
        b.init_state(1, ph, 1.0)
        for _ in range(n):
            b.step(1)
        assert np.array_equal(a.get_state(), b.get_state()), n
        a.close()
        b.close()


@pytest.mark.parametrize("cfg", [small(), small(prec=1), small(mode=1),
                                 dict(small(nx=40, ny=36), dim=3, nz=22, hz=0.2, lam=2.0, g=150.0)])
def test_restart_is_bitwise(P, cfg):
    """Stop after k steps, save the state to the host, restart a new handle
    from it: the continuation repeats the uninterrupted run bit for bit
    (imaginary time in both precisions, real time, 3D)."""
    announce(f"restart dim={cfg['dim']} prec={cfg['precision']} mode={cfg['mode']}")
    sp = W.solver_params(cfg)
    ph = W.phase_field(4, cfg["ny"], cfg["nx"])
    a = P.Solver(sp)
    a.init_state(1, ph, 1.0)
    a.step(150)
    ref = a.get_state()
    b = P.Solver(sp)
    b.init_state(1, ph, 1.0)
    b.step(37)
    mid = b.get_state()
    c = P.Solver(sp)
    c.set_state(mid)
    c.step(113)
    assert np.array_equal(c.get_state(), ref)
    for s in (a, b, c):
        s.close()


def test_prepare_steps_leaves_the_state(P, monkeypatch):
    """prepare_steps picks the plan (and the fused step's tile shape) and
    captures graphs without advancing the state; the prepared call then
    gives the same bits as an unprepared handle's with the same choices."""
    announce("prepare_steps")
    cfg = small()
    ph = W.phase_field(5, cfg["ny"], cfg["nx"])
    a = P.Solver(W.solver_params(cfg))
    a.init_state(1, ph, 1.0)
    s0 = a.get_state()
    a.prepare_steps(20)
    assert np.array_equal(a.get_state(), s0)
    assert a.observables()["step"] == 0
    a.step(20)
    # the same tile shape (the norm partials are summed per tile)
    monkeypatch.setenv("SSCN_FUSED_TILE", str([[32, 32], [32, 16], [16, 16]].index(a.solver_info()["fused_tile"])))
    b = P.Solver(W.solver_params(cfg))
    b.init_state(1, ph, 1.0)
    b.set_plan(a.solver_info()["plan"])
    b.step(20)
    assert np.array_equal(a.get_state(), b.get_state())
    a.close()
    b.close()


@pytest.mark.parametrize("plan", [1, 2])
def test_batch_graph_steps(P, plan):
    """Batched calls of n steps (graphs, any n) against one-step calls
    (direct launches), bitwise, and prepare_steps leaves the states."""
    announce(f"batch graph steps plan={plan}")
    cfgs = [small(nx=60 + 8 * t, ny=50 + 6 * t, g=40.0 + 10 * t, omega=0.3 + 0.1 * t) for t in range(3)]
    phs = [W.phase_field(10 + t, c["ny"], c["nx"]) for t, c in enumerate(cfgs)]
    for n in (2, 3, 20, 257):
        a = P.Batch(cfgs)
        b = P.Batch(cfgs)
        for bb in (a, b):
            bb.set_plan(plan)
            for k in range(3):
                bb.init_state(k, 1, phs[k], 1.0)
        s0 = [a.get_state(k) for k in range(3)]
        a.prepare_steps(n)
        assert all(np.array_equal(a.get_state(k), s0[k]) for k in range(3))
        a.step(n)
        for _ in range(n):
            b.step(1)
        for k in range(3):
            assert np.array_equal(a.get_state(k), b.get_state(k)), (n, k)
        a.close()
        b.close()


def test_nonfinite_state_is_reported(P):
    """A NaN or Inf in the state makes both observables calls return
    SSCN_ENONFINITE (the single-instance and the batched one)."""
    import torch
    announce("non-finite states")
    cfg = small()
    for bad in (np.nan, np.inf):
        s = P.Solver(W.solver_params(cfg))
        s.init_state(1, W.phase_field(6, cfg["ny"], cfg["nx"]), 1.0)
        st = s.get_state()
        st[cfg["ny"] // 2, cfg["nx"] // 3] = complex(bad, 0.0)
        s.set_state(st)
        with pytest.raises(P.SSCNError) as ei:
            s.observables()
        assert ei.value.code == -4
        o = s.observables(raise_nonfinite=False)  # still filled
        assert not np.isfinite(o["norm"])
        s.close()
        cfgs = [small(nx=50, ny=40), small(nx=44, ny=36, g=20.0)]
        b = P.Batch(cfgs)
        for k, c in enumerate(cfgs):
            b.init_state(k, 1, W.phase_field(7 + k, c["ny"], c["nx"]), 1.0)
        b.psi[1][5, 7] = complex(bad, 1.0)
        torch.cuda.synchronize()
        with pytest.raises(P.SSCNError) as ei:
            b.observables()
        assert ei.value.code == -4
        b.close()


def test_batch_criterion_equals_single_converge(P):
    """sscn_batch_run applies sscn_converge's criterion (|dmu| < tol at two
    consecutive checks with an unchanged vortex count) per instance on the
    device: each instance stops at the single-instance run's step (or one
    check away, where the two mu sums, reduced in different orders, fall on
    either side of tol) with the same vortex count."""
    announce("batched criterion vs sscn_converge")
    cfgs = [dict(dim=2, nx=64, ny=64, nz=1, hx=0.2, hy=0.2, hz=0.1, gamma=1.0, nu=1.0 + 0.05 * t, lam=1.0,
                 g=40.0 + 30.0 * t, omega=0.55 + 0.1 * t, dt=5e-3, mode=0, precision=0) for t in range(3)]
    phs = [W.phase_field(20 + t, 64, 64) for t in range(3)]
    K = 20
    b = P.Batch(cfgs)
    for k in range(3):
        b.init_state(k, 1, phs[k], 1.0)
    steps_b = b.run(max_steps=400000, check_every=K, tol=1e-8)
    for k, c in enumerate(cfgs):
        s = P.Solver(W.solver_params(c))
        s.init_state(1, phs[k], 1.0)
        steps_s, ok = s.converge(400000, check_every=K, tol=1e-8)
        assert ok and steps_b[k] > 0
        assert abs(steps_b[k] - steps_s) <= K, (k, steps_b[k], steps_s)
        if steps_b[k] == steps_s:
            assert np.array_equal(b.get_state(k), s.get_state()) or \
                float(np.linalg.norm(b.get_state(k) - s.get_state())) <= 1e-10
        assert b.vortex_count(k) == s.vortex_count(), k
        s.close()
    b.close()


def test_batch_profile_step(P):
    """The per-kernel profile of the batched step advances the batch like
    ordinary steps (checked against the oracle) and returns positive
    durations whose sum is within the step time."""
    announce("batch profile step")
    cfgs = [small(nx=80, ny=64), small(nx=64, ny=90, g=90.0)]
    b = P.Batch(cfgs)
    for k, c in enumerate(cfgs):
        b.init_state(k, 1, W.phase_field(30 + k, c["ny"], c["nx"]), 1.0)
    for plan in (1, 2):
        b.set_plan(plan)
        prof = b.profile_step(5)
        assert prof["step"] > 0
        if plan == 1:
            assert prof["x"] > 0 and prof["y"] > 0 and prof["x"] + prof["y"] <= prof["step"] * 1.0001
        else:
            assert 0 < prof["fused"] <= prof["step"] * 1.0001
    for k, c in enumerate(cfgs):
        op = O.make_params(**c)
        ref = O.step(op, O.init_state(op, 1, W.phase_field(30 + k, c["ny"], c["nx"]), 1.0), 10)
        got = b.get_state(k)
        assert float(np.linalg.norm(got - ref) / np.linalg.norm(ref)) <= 1e-10, k
    b.close()
