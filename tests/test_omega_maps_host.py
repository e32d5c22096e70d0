"""Host logic of the rotation maps (no GPU): grid sizing and the bisection
of Omega_c, with the batched runs replaced by a synthetic count rule."""
import math

import pytest

from paper_1906_06327_amd import omega_maps as M


def test_grid_side_holds_the_condensate_and_grows_with_g_and_omega():
    for g in (25.0, 100.0, 400.0):
        for om in (0.0, 0.5, 0.8):
            n = M.grid_side(g, om, 0.1)
            a = 1.0 - om * om
            mu = math.sqrt(g * a / math.pi)
            r = math.sqrt(2.0 * mu / a)
            assert n in M.SIZES
            assert n * 0.1 >= 2.8 * r or n == M.SIZES[-1]
    assert M.grid_side(100.0, 0.3, 0.1) <= M.grid_side(800.0, 0.3, 0.1)
    assert M.grid_side(100.0, 0.3, 0.1) <= M.grid_side(100.0, 0.9, 0.1)
    with pytest.raises(ValueError):
        M.grid_side(100.0, 1.0, 0.1)


def test_bracket_update():
    assert M.bracket_update(0.1, 0.9, 0.5, 0) == (0.5, 0.9)
    assert M.bracket_update(0.1, 0.9, 0.5, 3) == (0.1, 0.5)


def test_omega_c_bisection_finds_a_synthetic_threshold(monkeypatch):
    # a vortex survives above Omega_c(g) = 0.3 + 0.05 log10(g) + 0.01 seed'
    def true_oc(g, seed):
        return 0.3 + 0.05 * math.log10(g) + 0.01 * (seed - 13)

    calls = []

    def fake_run(specs, log=None, **_):
        calls.append(len(specs))
        return [{"g": s["g"], "omega": s["omega"], "seed": s["seed"],
                 "vortices": 1 if s["omega"] > true_oc(s["g"], s["seed"]) else 0} for s in specs]

    monkeypatch.setattr(M, "run_instances", fake_run)
    res = M.omega_c([50.0, 400.0], seeds=(13, 14, 15), lo=0.1, hi=0.9, rounds=8)
    assert calls == [6] * 8  # every (g, seed) pair in every round, one batch each
    for g, r in res.items():
        for (a, b), s in zip(r["brackets"], (13, 14, 15)):
            assert a <= true_oc(g, s) <= b and b - a == pytest.approx(0.8 / 2 ** 8)
        mean = sum(true_oc(g, s) for s in (13, 14, 15)) / 3
        assert abs(r["omega_c"] - mean) <= 0.8 / 2 ** 9 + 1e-12


def test_count_map_builds_the_full_grid(monkeypatch):
    seen = []

    def fake_run(specs, **_):
        seen.extend(specs)
        return [{"g": s["g"], "omega": s["omega"], "kind": s["kind"], "seed": s["seed"], "n": s["nx"]}
                for s in specs]

    monkeypatch.setattr(M, "run_instances", fake_run)
    recs = M.count_map([50.0, 800.0], [0.3, 0.7], kinds=(1, 0), seeds=(13, None), h=0.1, dt=1e-3)
    assert len(recs) == len(seen) == 2 * 2 * 2 * 2
    combos = {(s["g"], s["omega"], s["kind"], s["seed"]) for s in seen}
    assert len(combos) == 16
    for s in seen:
        assert s["dim"] == 2 and s["nx"] == s["ny"] == M.grid_side(s["g"], s["omega"], 0.1)
        assert s["hx"] == s["hy"] == 0.1 and s["dt"] == 1e-3 and s["mode"] == 0
    # a larger condensate gets a larger grid
    assert max(s["nx"] for s in seen if s["g"] == 800.0) >= max(s["nx"] for s in seen if s["g"] == 50.0)
