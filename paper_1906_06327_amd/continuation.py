"""Continuation start: the paper's chain of vortex lattices.

Sec. 3 of the paper converges the lattice of larger nonlinearity and/or
rotation from the converged state of smaller ones rather than from the
one-vortex random-phase state of Eq. (fun), on a grid enlarged to hold the
larger condensate (the old grid is read into the centre of the new one).
Fig. 2 and Table 1 chain four 2D lattices this way, with h = 0.05 and
Delta = 0.00025 in imaginary time:

    (a) g = 100, Omega = 0.8,   257 x 257 points,  7 vortices, from Eq. (fun)
    (b) g = 100, Omega = 0.95,  321 x 321 points, 19 vortices, from (a)
    (c) g = 500, Omega = 0.92,  401 x 401 points, 37 vortices, from (b)
    (d) g = 500, Omega = 0.978, 441 x 441 points, 61 vortices, from (c)

This module runs that chain on the library's kernels: `sscn_embed_state`
places each converged state at the centre of the next grid (the library
stores n points per axis, the paper's n + 1 minus its always-zero last
row), and `sscn_converge` runs imaginary time to |mu_n - mu_{n-1}| < tol at
two consecutive checks 0.1 time units apart with an unchanged vortex count.
With `npas` every lattice instead runs the paper's fixed number of steps
(NPAS, 3 x 10^6 in the paper's programs), with mu, E and the vortex count
recorded at checkpoints.  With `scratch` the lattices (b)-(d) are also run
from Eq. (fun) for comparison (Fig. 3 of the paper: 12 x 10^5 steps against
30 000 for (b)).
"""
import argparse
import json
import time

from . import Solver, embed_state, SSCN_IMAG, SSCN_C128

H = 0.05
DT = 2.5e-4
# (g, Omega, stored points per axis, vortices the paper reports)
CHAIN = ((100.0, 0.8, 256, 7), (100.0, 0.95, 320, 19), (500.0, 0.92, 400, 37), (500.0, 0.978, 440, 61))


# The 3D chain of Fig. 5 / Table 1: lambda = 100, h_z = 0.025, 33 points in
# z (32 stored), g_3D = g_2D sqrt(2 pi / lambda), and (d) on 451 x 451 points.
LAM_3D, HZ_3D, NZ_3D = 100.0, 0.025, 32
CHAIN_3D = ((25.0662827, 0.8, 256, 7), (25.0662827, 0.95, 320, 19), (125.33141, 0.92, 400, 37),
            (125.33141, 0.978, 450, 61))


def params(g, omega, n, dim=2, precision=SSCN_C128):
    if dim == 3:
        return dict(dim=3, nx=n, ny=n, nz=NZ_3D, hx=H, hy=H, hz=HZ_3D, gamma=1.0, nu=1.0, lam=LAM_3D, g=g,
                    omega=omega, dt=DT, mode=SSCN_IMAG, precision=precision)
    return dict(dim=2, nx=n, ny=n, nz=1, hx=H, hy=H, hz=0.1, gamma=1.0, nu=1.0, lam=1.0, g=g,
                omega=omega, dt=DT, mode=SSCN_IMAG, precision=precision)


def _converge(torch, s, max_steps, tol):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, ok = s.converge(max_steps, check_every=int(round(0.1 / DT)), tol=tol)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    o = s.observables()
    return {"steps": steps if ok else -1, "steps_run": steps, "converged": ok, "wall_s": round(wall, 3),
            "mu": o["mu"], "energy": o["energy"], "mu_full": o["mu_full"],
            "energy_full": o["energy_full"], "vortices": s.vortex_count()}


def _fixed(torch, s, npas, every, settle):
    """The paper's procedure: a fixed number of steps (NPAS).  Records mu,
    E and the vortex count every `every` steps and the first checkpoint
    from which mu stays within `settle` of its final value."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist, done = [], 0
    while done < npas:
        k = min(every, npas - done)
        s.step(k)
        done += k
        o = s.observables()
        hist.append((done, o["mu"], o["energy"], s.vortex_count()))
    wall = time.perf_counter() - t0
    o = s.observables()
    mu_end = hist[-1][1]
    settled = hist[-1][0]
    for step, mu, _, _ in reversed(hist):
        if abs(mu - mu_end) > settle:
            break
        settled = step
    return {"steps": npas, "wall_s": round(wall, 3), "mu": o["mu"], "energy": o["energy"],
            "mu_full": o["mu_full"], "energy_full": o["energy_full"], "vortices": s.vortex_count(),
            "settled_within": settle, "settled_step": settled,
            "history": [(st, round(mu, 7), round(e, 7), v) for st, mu, e, v in hist]}


def run_chain(max_steps=2000000, tol=1e-8, seed=13, scratch=False, scratch_steps=3000000, log=print,
              chain=CHAIN, npas=0, every=50000, settle=1e-4, save=None, dim=2, precision=SSCN_C128,
              npas_next=0):
    """Converge the chain; returns one record per lattice (continuation
    start from the previous lattice, and with `scratch` from Eq. (fun))."""
    import torch
    import workloads as W
    out, prev = [], None
    for k, (g, omega, n, nv) in enumerate(chain):
        s = Solver(params(g, omega, n, dim, precision))
        if prev is None:
            s.init_state(1, W.phase_field(seed, n, n), 1.0)
            start = "Eq. (fun)"
        else:
            embed_state(prev.psi, s.psi)
            s.set_state_device()
            start = f"lattice {chain[k - 1][:2]} embedded {chain[k - 1][2]} -> {n}"
        rec = {"g": g, "omega": omega, "n": n, "paper_vortices": nv, "start": start}
        nfix = npas_next if (prev is not None and npas_next > 0) else npas
        run = (lambda sv, cap: _fixed(torch, sv, nfix, every, settle)) if npas > 0 else \
              (lambda sv, cap: _converge(torch, sv, cap, tol))
        rec.update(run(s, max_steps))
        if log:
            log(f"[continuation] g={g} Omega={omega} n={n}: {rec['steps']} steps, "
                f"{rec['wall_s']} s, mu {rec['mu']:.6f}, E {rec['energy']:.6f}, {rec['vortices']} vortices"
                + (f", mu settled to {settle:g} at step {rec['settled_step']}" if npas > 0 else ""))
        if scratch and prev is not None:
            s0 = Solver(params(g, omega, n, dim, precision))
            s0.init_state(1, W.phase_field(seed, n, n), 1.0)
            rec["from_fun"] = run(s0, scratch_steps)
            s0.close()
            if log:
                f = rec["from_fun"]
                log(f"[continuation]   from Eq. (fun): {f['steps']} steps, {f['wall_s']} s, "
                    f"mu {f['mu']:.6f}, {f['vortices']} vortices"
                    + (f", mu settled at step {f['settled_step']}" if npas > 0 else ""))
        if save:
            import numpy as np
            np.save(f"{save}/lattice{dim}d_g{g:g}_omega{omega:g}_n{n}.npy", s.get_state())
        if prev is not None:
            prev.close()
        prev = s
        out.append(rec)
    prev.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--max-steps", type=int, default=2000000)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--seed", type=int, default=13)
    ap.add_argument("--scratch", action="store_true", help="also converge (b)-(d) from Eq. (fun)")
    ap.add_argument("--scratch-steps", type=int, default=3000000)
    ap.add_argument("--npas", type=int, default=0,
                    help="run this fixed number of steps per lattice (the paper's NPAS) instead of "
                         "stopping at the convergence criterion")
    ap.add_argument("--every", type=int, default=50000, help="checkpoint interval with --npas")
    ap.add_argument("--settle", type=float, default=1e-4, help="mu band for the settled step with --npas")
    ap.add_argument("--save-states", default=None, help="directory for each lattice's final state (.npy)")
    ap.add_argument("--lattices", type=int, default=len(CHAIN), help="run only the first k lattices")
    ap.add_argument("--npas-next", type=int, default=0,
                    help="with --npas: steps for the continued lattices (default: --npas)")
    ap.add_argument("--dim", type=int, default=2, choices=(2, 3), help="the 2D chain of Fig. 2 or the 3D one of Fig. 5")
    ap.add_argument("--c64", action="store_true", help="complex64 sweeps (FP64 reductions)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    chain = CHAIN if a.dim == 2 else CHAIN_3D
    res = run_chain(a.max_steps, a.tol, a.seed, a.scratch, a.scratch_steps, npas=a.npas, every=a.every,
                    settle=a.settle, save=a.save_states, chain=chain[:a.lattices], dim=a.dim,
                    precision=1 if a.c64 else SSCN_C128, npas_next=a.npas_next)
    text = json.dumps({"h": H, "dt": DT, "tol": a.tol, "npas": a.npas, "chain": res}, indent=1)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text + "\n")
    print(text, flush=True)


if __name__ == "__main__":
    main()
