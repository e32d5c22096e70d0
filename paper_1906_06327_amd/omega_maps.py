"""Vortex count against rotation, and the critical rotation of the first vortex.

Sec. 4 of the paper maps how many vortices imaginary time converges to as
the rotation Omega grows at fixed nonlinearity g_2D (Figs. 2 and 4), and
measures the critical rotation Omega_c(g_2D) above which the one-vortex
start of Eq. (fun), with its random phase, keeps a vortex and below which
it ends vortex-free (Fig. 1, averaged over several random phases).

Both maps here are batched runs of the library (`sscn_batch_*`): one
imaginary-time instance per (g, Omega, start, seed), advanced together by
the fused batched step until every instance has |mu_n - mu_{n-1}| < tol at
two consecutive checks (or max_steps), then counted (`sscn_batch_vortex_count`).

- `count_map` runs a grid of Omega values for each g.
- `omega_c` bisects Omega_c for every (g, seed) pair at once: each round is
  one batch holding every pair at the midpoint of its bracket, and the
  count there (zero or not) halves the bracket.  The estimate is the final
  bracket's midpoint, averaged over the seeds as in Fig. 1.

The batched criterion has no vortex-count condition, so an instance on one
of the plateaus of Fig. 3 can stop there; near Omega_c the approach is
slow, and an instance that has not converged within max_steps is counted
as it stands (the paper's fixed NPAS does the same).
"""
import argparse
import json
import math
import time

from . import Batch, SSCN_IMAG, SSCN_C128

SIZES = (128, 160, 192, 256, 320, 384, 512)
MAX_BATCH = 64


def grid_side(g, omega, h, gamma=1.0, nu=1.0, sizes=SIZES):
    """Smallest stored side n (from `sizes`) whose extent n h holds 2 x 1.4
    Thomas-Fermi radii of the rotating condensate: mu = sqrt(g (gamma^2 -
    Omega^2)^(1/2) (nu^2 - Omega^2)^(1/2) / pi) and R = sqrt(2 mu) /
    sqrt(gamma^2 - Omega^2) (the largest size if none does)."""
    a = gamma * gamma - omega * omega
    b = nu * nu - omega * omega
    if a <= 0.0 or b <= 0.0:
        raise ValueError("Omega must stay below both trap frequencies")
    mu = math.sqrt(g * math.sqrt(a * b) / math.pi)
    r = math.sqrt(2.0 * mu) / math.sqrt(min(a, b))
    for n in sizes:
        if n * h >= 2.0 * 1.4 * r:
            return n
    return sizes[-1]


def instance(g, omega, h=0.1, dt=1e-3, gamma=1.0, nu=1.0, n=None):
    n = n or grid_side(g, omega, h, gamma, nu)
    return dict(dim=2, nx=n, ny=n, nz=1, hx=h, hy=h, hz=h, gamma=gamma, nu=nu, lam=1.0, g=float(g),
                omega=float(omega), dt=dt, mode=SSCN_IMAG, precision=SSCN_C128)


def run_instances(specs, max_steps=2_000_000, check_every=100, tol=1e-8, log=None):
    """specs: dicts with the solver parameters plus `kind` (1 one vortex, 0
    Gaussian) and `seed` (None: no random phase).  Runs them in batches of
    at most 64 and returns one record per spec, in order."""
    import workloads as W
    out = []
    for b0 in range(0, len(specs), MAX_BATCH):
        part = specs[b0:b0 + MAX_BATCH]
        keys = ("dim", "nx", "ny", "nz", "hx", "hy", "hz", "gamma", "nu", "lam", "g", "omega", "dt", "mode",
                "precision")
        b = Batch([{k: s[k] for k in keys} for s in part])
        try:
            for k, s in enumerate(part):
                ph = W.phase_field(s["seed"], s["ny"], s["nx"]) if s.get("seed") is not None else None
                b.init_state(k, s.get("kind", 1), ph, s.get("d_xy", 1.0))
            t0 = time.perf_counter()
            steps = b.run(max_steps, check_every, tol)
            wall = time.perf_counter() - t0
            obs = b.observables()
            for k, s in enumerate(part):
                out.append({"g": s["g"], "omega": s["omega"], "n": s["nx"], "kind": s.get("kind", 1),
                            "seed": s.get("seed"), "converged": steps[k] >= 0,
                            "steps": steps[k] if steps[k] >= 0 else int(obs[k]["step"]),
                            "mu": obs[k]["mu"], "vortices": b.vortex_count(k)})
            if log:
                log(f"[omega_maps] batch of {len(part)}: {wall:.1f} s, "
                    f"{sum(1 for v in steps if v >= 0)} converged")
        finally:
            b.close()
    return out


def count_map(g_list, omegas, kinds=(1,), seeds=(13,), h=0.1, dt=1e-3, **run):
    """Vortex count on a grid of (g, Omega, start, seed)."""
    specs = [dict(instance(g, om, h, dt), kind=kd, seed=sd)
             for g in g_list for om in omegas for kd in kinds for sd in seeds]
    return run_instances(specs, **run)


def bracket_update(lo, hi, mid, vortices):
    """One bisection step for Omega_c: a vortex at mid moves the upper end
    there, none moves the lower end."""
    return (lo, mid) if vortices > 0 else (mid, hi)


def omega_c(g_list, seeds=(13, 14, 15), lo=0.1, hi=0.9, rounds=6, h=0.1, dt=1e-3, log=None, **run):
    """Omega_c(g) by bisection of every (g, seed) pair in parallel; returns
    {g: {"omega_c": mean over seeds, "per_seed": [...], "bracket": ...}}."""
    br = {(g, s): (lo, hi) for g in g_list for s in seeds}
    for r in range(rounds):
        pairs = list(br)
        specs = [dict(instance(g, 0.5 * (br[(g, s)][0] + br[(g, s)][1]), h, dt), kind=1, seed=s)
                 for g, s in pairs]
        recs = run_instances(specs, log=log, **run)
        for (g, s), rec in zip(pairs, recs):
            br[(g, s)] = bracket_update(*br[(g, s)], rec["omega"], rec["vortices"])
        if log:
            log(f"[omega_maps] round {r + 1}/{rounds}: " +
                ", ".join(f"g={g:g} s={s}: [{a:.4f}, {b:.4f}]" for (g, s), (a, b) in sorted(br.items())))
    res = {}
    for g in g_list:
        est = [0.5 * sum(br[(g, s)]) for s in seeds]
        res[g] = {"omega_c": sum(est) / len(est), "per_seed": est,
                  "brackets": [br[(g, s)] for s in seeds]}
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("what", choices=("counts", "omega_c"))
    ap.add_argument("--g", type=float, nargs="+", default=[100.0])
    ap.add_argument("--omegas", type=float, nargs="+", default=[0.3, 0.4, 0.5, 0.6, 0.7, 0.8])
    ap.add_argument("--seeds", type=int, nargs="+", default=[13])
    ap.add_argument("--gaussian", action="store_true", help="count map: also the Gaussian start")
    ap.add_argument("--rounds", type=int, default=6)
    ap.add_argument("--h", type=float, default=0.1)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--max-steps", type=int, default=2_000_000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    run = dict(max_steps=a.max_steps)
    if a.what == "counts":
        res = count_map(a.g, a.omegas, kinds=(1, 0) if a.gaussian else (1,), seeds=a.seeds, h=a.h, dt=a.dt,
                        log=print, **run)
    else:
        res = omega_c(a.g, seeds=a.seeds, rounds=a.rounds, h=a.h, dt=a.dt, log=print, **run)
        res = {str(k): v for k, v in res.items()}
    text = json.dumps(res, indent=1)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text + "\n")
    print(text, flush=True)


if __name__ == "__main__":
    main()
