"""Learned initial state for imaginary-time runs.

The paper shortens imaginary-time runs by starting from a better state than
the one-vortex random-phase state of Eq. (fun): a converged state of nearby
parameters (Sec. 3, Fig. 3).  Here a U-Net (paper_1906_06327_amd/nn.py)
learns that map from converged states the batched solver produces itself:

1. generate: draw (Omega, g, nu), converge each instance from Eq. (fun)
   with the batched fused step (sscn_batch_run), keep the state and its
   images under the symmetries of the rotating problem (rotation by pi, and
   each axis reflection combined with complex conjugation);
2. train: Adam on the phase-aligned loss against the nearest image, forward
   and backward on the bf16 matrix-core kernels of include/sscn_nn.h;
3. propose: the network's output, written into each instance's buffer,
   walls zeroed and normalised (sscn_batch_set_state_device);
4. evaluate: steps and wall time to |mu_n - mu_{n-1}| < tol from the learned
   start and from Eq. (fun), and the vortex counts of both results.

Every instance uses a grid of n x n points scaled to its Thomas-Fermi size:
with trap frequencies reduced by rotation, a = gamma^2 - Omega^2 and
b = nu^2 - Omega^2, the 2D Thomas-Fermi chemical potential is
mu = sqrt(g sqrt(a b) / pi) and the long radius R = sqrt(2 mu / a); the grid
spans 2 * BOX * R, so the coordinates x / (BOX R) of grid points are the
same for every instance and the network needs no resampling.
"""
import argparse
import json
import math
import time

import numpy as np

from . import Batch
from . import nn

BOX = 1.35
N_GRID = 128
CHANS = (32, 64, 128, 256, 256)
BOTT = 256
RANGES = dict(omega=(0.5, 0.9), g=(100.0, 1000.0), nu=(1.0, 1.2))


def tf_instance(omega, g, nu, n=N_GRID, dt=2e-3, precision=0, box=BOX):
    """Solver parameters of one instance on its Thomas-Fermi-scaled grid."""
    a = 1.0 - omega * omega
    b = nu * nu - omega * omega
    if a <= 0 or b <= 0:
        raise ValueError("Omega must stay below both trap frequencies")
    mu = math.sqrt(g * math.sqrt(a * b) / math.pi)
    r = math.sqrt(2.0 * mu / a)
    h = 2.0 * box * r / n
    return dict(dim=2, nx=n, ny=n, nz=1, hx=h, hy=h, hz=h, gamma=1.0, nu=nu, lam=1.0, g=g,
                omega=omega, dt=dt, mode=0, precision=precision)


def draw(m, seed, ranges=RANGES):
    """m parameter triples (Omega, g, nu): Omega and nu uniform, g log-uniform."""
    rng = np.random.default_rng(int(seed))
    out = []
    for _ in range(m):
        om = float(rng.uniform(*ranges["omega"]))
        g = float(math.exp(rng.uniform(math.log(ranges["g"][0]), math.log(ranges["g"][1]))))
        nu = float(rng.uniform(*ranges["nu"]))
        out.append((om, g, nu))
    return out


def features(plist, n=N_GRID):
    """Network input (B, n, n, 16) fp32: x/(BOX R), y/(BOX R), and Omega, log g,
    nu centred and scaled over their ranges; channels 5..15 zero."""
    ax = (np.arange(n) - n / 2) * 2.0 / n
    X, Y = np.meshgrid(ax, ax)
    lg0 = 0.5 * (math.log(RANGES["g"][0]) + math.log(RANGES["g"][1]))
    lgs = 0.5 * (math.log(RANGES["g"][1]) - math.log(RANGES["g"][0]))
    f = np.zeros((len(plist), n, n, nn.IN_CH), np.float32)
    for k, (om, g, nu) in enumerate(plist):
        f[k, ..., 0] = X
        f[k, ..., 1] = Y
        f[k, ..., 2] = (om - 0.7) / 0.2
        f[k, ..., 3] = (math.log(g) - lg0) / lgs
        f[k, ..., 4] = (nu - 1.1) / 0.1
    return f


def images(psi):
    """psi and its images under rotation by pi, conj(psi(-x, y)) and
    conj(psi(x, -y)); on the grid x_i = -n h / 2 + i h the reflection is
    the index map i -> (n - i) mod n."""
    n = psi.shape[0]
    r = (-np.arange(n)) % n
    return [psi, psi[r][:, r], np.conj(psi[:, r]), np.conj(psi[r, :])]


def target_scale(p):
    """Targets are psi * h * n / 4 (mean |psi|^2 over the grid 1/16)."""
    return p["hx"] * p["nx"] / 4.0


def _bf16_device(torch, a):
    t32 = torch.tensor(a, dtype=torch.float32, device="cuda")
    out = torch.empty(a.shape, dtype=torch.int16, device="cuda")
    nn.f32_to_bf16(t32, out)
    return out


def _run_logged(b, max_steps, chk, tol, log, tag, seg=100000):
    """sscn_batch_run in segments (the run resumes exactly where it stopped),
    with a progress line after each."""
    K = chk + (chk & 1)
    seg = max(K, seg // K * K)
    done, steps = 0, [-1] * b.n
    while done < max_steps:
        m = min(seg, max_steps - done)
        steps = b.run(m, check_every=chk, tol=tol)
        done += m
        nconv = sum(1 for s in steps if s >= 0)
        if log:
            log(f"[{tag}] {done} steps: {nconv}/{b.n} converged")
        if nconv == b.n:
            break
    return steps


def _run_batch(torch, plist, dt, max_steps, tol, seeds, starts=None, precision=0, log=None, tag="run"):
    """One batch from Eq. (fun) (starts None) or from proposed states."""
    n = N_GRID
    ps = [tf_instance(*p, n=n, dt=dt, precision=precision) for p in plist]
    b = Batch(ps)
    import workloads as W
    t0 = time.perf_counter()
    for k in range(len(ps)):
        if starts is None:
            b.init_state(k, 1, W.phase_field(seeds[k], n, n), 1.0)
        else:
            nn.f32_to_psi(starts[k], nn.OUT_CH, n * n, 1.0, b.psi[k])
            b.set_state_device(k)
    chk = max(2, int(round(0.1 / dt)))
    steps = _run_logged(b, max_steps, chk, tol, log, tag)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    obs = b.observables()
    counts = [b.vortex_count(k) for k in range(len(ps))]
    return b, ps, steps, wall, obs, counts


def generate(plist, seeds, dt=2e-3, max_steps=250000, tol=1e-6, chunk=64, log=print):
    """Converged states of plist (host complex128 list) plus run records."""
    import torch
    states, recs = [], []
    for c0 in range(0, len(plist), chunk):
        pl = plist[c0:c0 + chunk]
        b, ps, steps, wall, obs, counts = _run_batch(torch, pl, dt, max_steps, tol, seeds[c0:c0 + chunk],
                                                     log=log, tag="generate")
        for k in range(len(pl)):
            states.append(b.get_state(k))
            recs.append(dict(params=pl[k], steps=steps[k], mu=obs[k]["mu"], vortices=counts[k],
                             h=ps[k]["hx"]))
        b.close()
        done = sum(1 for s in steps if s > 0)
        log(f"[generate] {c0 + len(pl)}/{len(plist)}: {wall:.1f} s, {done}/{len(pl)} reached tol {tol:g}")
    return states, recs


def make_targets(plist, states, dt=2e-3):
    """(M, 4, n, n, 2) fp32 targets: the scaled state and its three images."""
    n = N_GRID
    T = np.zeros((len(states), 4, n, n, 2), np.float32)
    for m, (p, s) in enumerate(zip(plist, states)):
        sc = target_scale(tf_instance(*p, n=n, dt=dt))
        for k, im in enumerate(images(s)):
            T[m, k, ..., 0] = im.real * sc
            T[m, k, ..., 1] = im.imag * sc
    return T


def train(net, X, T, epochs, lr=1e-3, seed=0, log=print, log_every=50, warmup=0, clip=0.0):
    """Adam over shuffled minibatches of net.N samples with a cosine
    learning-rate decay after a linear warm-up over the first `warmup`
    iterations.  clip > 0 bounds the global gradient norm of every step by
    clip times a running average of the (clipped) norms of the earlier
    steps, so that a single outlying batch cannot throw the weights far.
    X: (M, n, n, 16) bf16 device tensor; T: (M, 4, n, n, 2) fp32 device
    tensor.  Returns the per-epoch mean loss."""
    import torch
    M, B = X.shape[0], net.N
    per = M // B
    total = max(1, epochs * per)
    rng = np.random.default_rng(seed)
    hist, it = [], 0
    gavg, nclip = None, 0
    for ep in range(epochs):
        perm = rng.permutation(M)
        acc = 0.0
        for s in range(per):
            idx = torch.tensor(perm[s * B:(s + 1) * B], device="cuda")
            net.forward(X.index_select(0, idx))
            lv = float(net.loss_and_grad(T.index_select(0, idx)).mean())
            net.backward(net.gacts["out"])
            ramp = min(1.0, (it + 1) / warmup) if warmup > 0 else 1.0
            step_lr = lr * ramp * 0.5 * (1.0 + math.cos(math.pi * it / total))
            if clip > 0:
                gsq = net.grad_sqnorm()
                bound = clip * gavg if gavg is not None else None
                net.adam_step(lr=step_lr, max_norm=bound, gsq=gsq)
                gn = math.sqrt(float(gsq[0]))
                if bound is not None and gn > bound:
                    nclip += 1
                    gn = bound
                gavg = gn if gavg is None else 0.98 * gavg + 0.02 * gn
            else:
                net.adam_step(lr=step_lr)
            acc += lv
            it += 1
            if log_every and it % log_every == 0:
                extra = f" grad norm avg {gavg:.4g}, {nclip} clipped" if clip > 0 else ""
                log(f"[train] iter {it}/{total} loss {lv:.4f}{extra}")
        hist.append(acc / max(1, per))
        log(f"[train] epoch {ep + 1}/{epochs} mean loss {hist[-1]:.4f}")
    return hist


def propose(net_params, plist, chans=CHANS, bott=BOTT):
    """Network output (B, n, n, 16) fp32 device tensor for plist."""
    import torch
    net = nn.UNet(len(plist), N_GRID, N_GRID, chans=chans, bott=bott, params=net_params)
    X = _bf16_device(torch, features(plist))
    out = net.forward(X).clone()
    return out


def plain_runs(plist, seeds, dt=2e-3, max_steps=2000000, tol=1e-8, log=print):
    """The plain method: every instance alone from Eq. (fun), one after the
    other (the same kernels and criterion as a batch of one)."""
    import torch
    steps, walls, counts, mus = [], [], [], []
    for k, p in enumerate(plist):
        b, ps, st, wall, obs, cnt = _run_batch(torch, [p], dt, max_steps, tol, [seeds[k]], log=None)
        b.close()
        steps.append(st[0])
        walls.append(wall)
        counts.append(cnt[0])
        mus.append(obs[0]["mu"])
        log(f"[plain] instance {k + 1}/{len(plist)}: {st[0]} steps, {wall:.2f} s")
    return steps, walls, counts, mus


def evaluate(net_params, plist, seeds, dt=2e-3, max_steps=2000000, tol=1e-8, plain=False, log=print,
             chans=CHANS, bott=BOTT):
    """The learned start and Eq. (fun) to |dmu| < tol on the same GPU, one
    batch each; with plain, also every instance alone from Eq. (fun)."""
    import torch
    res_plain = plain_runs(plist, seeds, dt, max_steps, tol, log) if plain else None
    b, ps, st0, wall0, obs0, cnt0 = _run_batch(torch, plist, dt, max_steps, tol, seeds, log=log,
                                               tag="one-vortex start")
    finals = [b.get_state(k) for k in range(len(plist))]
    b.close()
    log(f"[evaluate] one-vortex start: {wall0:.1f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    starts = propose(net_params, plist, chans, bott)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    b, ps, st1, wall1, obs1, cnt1 = _run_batch(torch, plist, dt, max_steps, tol, seeds, starts=starts, log=log,
                                               tag="learned start")
    b.close()
    # distance of each start from the state the one-vortex run converged to
    d_learned, d_fun = [], []
    import workloads as W
    pred = starts[..., :2].cpu().numpy().astype(np.float64)
    b0 = Batch([tf_instance(*p, n=N_GRID, dt=dt) for p in plist])
    for k in range(len(plist)):
        b0.init_state(k, 1, W.phase_field(seeds[k], N_GRID, N_GRID), 1.0)
        z = pred[k, ..., 0] + 1j * pred[k, ..., 1]
        z[0, :] = 0
        z[:, 0] = 0
        d_learned.append(phase_distance(z, finals[k]))
        d_fun.append(phase_distance(b0.get_state(k), finals[k]))
    b0.close()
    log(f"[evaluate] learned start: inference {t_inf:.2f} s + run {wall1:.1f} s")
    st0a, st1a = np.array(st0), np.array(st1)
    rows = []
    for k in range(len(plist)):
        rows.append(dict(omega=plist[k][0], g=plist[k][1], nu=plist[k][2],
                         distance_learned=round(d_learned[k], 5), distance_one_vortex=round(d_fun[k], 5),
                         steps_one_vortex=int(st0[k]), steps_learned=int(st1[k]),
                         vortices_one_vortex=cnt0[k], vortices_learned=cnt1[k],
                         mu_one_vortex=obs0[k]["mu"], mu_learned=obs1[k]["mu"]))
    both = (st0a > 0) & (st1a > 0)
    extra = {}
    if res_plain is not None:
        pst, pwall, pcnt, pmu = res_plain
        for k, r in enumerate(rows):
            r["steps_plain"] = int(pst[k])
            r["wall_plain_s"] = round(pwall[k], 3)
        extra = dict(wall_plain_s=round(sum(pwall), 3),
                     plain_steps_equal_batched=int(sum(1 for k in range(len(plist)) if pst[k] == st0[k])),
                     speedup_learned_batched_vs_plain=round(sum(pwall) / (wall1 + t_inf), 3),
                     speedup_batched_vs_plain=round(sum(pwall) / wall0, 3))
    return dict(
        instances=len(plist), tol=tol, dt=dt, grid=N_GRID,
        wall_one_vortex_s=round(wall0, 3), wall_learned_s=round(wall1 + t_inf, 3),
        inference_s=round(t_inf, 3),
        wall_speedup=round(wall0 / (wall1 + t_inf), 3),
        converged_one_vortex=int((st0a > 0).sum()), converged_learned=int((st1a > 0).sum()),
        median_steps_one_vortex=float(np.median(np.where(st0a > 0, st0a, max_steps))),
        median_steps_learned=float(np.median(np.where(st1a > 0, st1a, max_steps))),
        max_steps_one_vortex=int(np.where(st0a > 0, st0a, max_steps).max()),
        max_steps_learned=int(np.where(st1a > 0, st1a, max_steps).max()),
        same_vortex_count=int(sum(1 for r in rows if r["vortices_one_vortex"] == r["vortices_learned"])),
        lower_or_equal_mu_learned=int(sum(1 for r in rows if r["mu_learned"] <= r["mu_one_vortex"] + 1e-7)),
        both_converged=int(both.sum()),
        median_distance_learned=round(float(np.median(d_learned)), 5),
        median_distance_one_vortex=round(float(np.median(d_fun)), 5),
        total_steps_both_converged_one_vortex=int(st0a[both].sum()),
        total_steps_both_converged_learned=int(st1a[both].sum()),
        learned_fewer_steps=int((st1a[both] < st0a[both]).sum()),
        **extra,
        rows=rows)


def tf_instance_3d(omega, g2d, nu, lam, nz, hz, n=N_GRID, dt=2e-3, precision=0):
    """3D parameters whose x-y grid is the Thomas-Fermi-scaled grid of the 2D
    instance (Omega, g2d, nu): trap lam in z, nz points of spacing hz, and the
    3D nonlinearity g2d sqrt(2 pi / lam) of the quasi-2D reduction of Sec. 2
    (g_2D = g_3D sqrt(lam / (2 pi)))."""
    p = tf_instance(omega, g2d, nu, n=n, dt=dt, precision=precision)
    return dict(p, dim=3, nz=nz, hz=hz, lam=lam, g=g2d * math.sqrt(2.0 * math.pi / lam))


def evaluate_3d(net_params, plist, seeds, lam=100.0, nz=16, hz=0.05, dt=2e-3, max_steps=1000000, tol=1e-8,
                log=print, chans=CHANS, bott=BOTT):
    """The learned start in 3D: the 2D network's state for (Omega, g_2D, nu),
    normalised on its grid, times the normalised Gaussian of width
    1 / sqrt(lam) in z (the product form of Eq. (fun), sscn_extend_z), against
    Eq. (fun) itself; each instance alone on its 3D handle, to the same
    criterion."""
    import torch
    import workloads as W
    from . import Solver, extend_z
    n, d_z = N_GRID, 1.0 / math.sqrt(lam)
    chk = max(2, int(round(0.1 / dt)))
    rows = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    starts = propose(net_params, plist, chans, bott)
    b2 = Batch([tf_instance(*p, n=n, dt=dt) for p in plist])
    for k in range(len(plist)):
        nn.f32_to_psi(starts[k], nn.OUT_CH, n * n, 1.0, b2.psi[k])
        b2.set_state_device(k)  # walls zeroed, normalised on the 2D grid
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    for k, (om, g, nu) in enumerate(plist):
        p3 = tf_instance_3d(om, g, nu, lam, nz, hz, n=n, dt=dt)
        rec = dict(omega=om, g_2d=g, g_3d=p3["g"], nu=nu)
        for tag in ("one_vortex", "learned"):
            s = Solver(p3)
            log(f"[evaluate_3d] {k + 1}/{len(plist)} {tag} start: converging")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if tag == "one_vortex":
                s.init_state(1, W.phase_field(seeds[k], n, n), 1.0, d_z)
            else:
                extend_z(b2.psi[k], s.psi, hz, d_z)
                s.set_state_device()
            steps, ok = s.converge(max_steps, check_every=chk, tol=tol)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t1
            o = s.observables()
            rec.update({f"steps_{tag}": steps if ok else -1, f"wall_{tag}_s": round(wall, 3),
                        f"mu_{tag}": o["mu"], f"vortices_{tag}": s.vortex_count()})
            s.close()
        rows.append(rec)
        log(f"[evaluate_3d] {k + 1}/{len(plist)} Omega={om:.3f} g2D={g:.0f}: Eq. (fun) "
            f"{rec['steps_one_vortex']} steps {rec['wall_one_vortex_s']} s {rec['vortices_one_vortex']} vortices; "
            f"learned {rec['steps_learned']} steps {rec['wall_learned_s']} s {rec['vortices_learned']} vortices")
    b2.close()
    s0 = np.array([r["steps_one_vortex"] for r in rows])
    s1 = np.array([r["steps_learned"] for r in rows])
    both = (s0 > 0) & (s1 > 0)
    w0 = sum(r["wall_one_vortex_s"] for r in rows)
    w1 = sum(r["wall_learned_s"] for r in rows) + t_inf
    return dict(instances=len(plist), lam=lam, nz=nz, hz=hz, dt=dt, tol=tol, grid=n,
                inference_and_setup_s=round(t_inf, 3), wall_one_vortex_s=round(w0, 3), wall_learned_s=round(w1, 3),
                wall_speedup=round(w0 / w1, 3),
                converged_one_vortex=int((s0 > 0).sum()), converged_learned=int((s1 > 0).sum()),
                both_converged=int(both.sum()),
                total_steps_both_converged_one_vortex=int(s0[both].sum()),
                total_steps_both_converged_learned=int(s1[both].sum()),
                learned_fewer_steps=int((s1[both] < s0[both]).sum()),
                same_vortex_count=int(sum(1 for r in rows if r["vortices_one_vortex"] == r["vortices_learned"])),
                rows=rows)


def phase_distance(a, b):
    """min over phi of |a/|a| - e^{i phi} b/|b||: sqrt(2 - 2 |<a, b>|) for
    unit vectors (0 = the same state up to a global phase, sqrt 2 =
    orthogonal)."""
    a = a / np.linalg.norm(a)
    b = b / np.linalg.norm(b)
    return float(np.sqrt(max(0.0, 2.0 - 2.0 * abs(np.vdot(b, a)))))


def save_params(path, params):
    np.savez(path, **{f"{k}__w": v[0] for k, v in params.items()}, **{f"{k}__b": v[1] for k, v in params.items()})


def load_params(path):
    d = np.load(path)
    names = sorted({k.rsplit("__", 1)[0] for k in d.files})
    return {k: (d[f"{k}__w"], d[f"{k}__b"]) for k in names}


def main(argv=None):
    ap = argparse.ArgumentParser(description="Generate, train and evaluate the learned initial state.")
    ap.add_argument("--train", type=int, default=1024, help="training instances")
    ap.add_argument("--eval", type=int, default=64, help="held-out evaluation instances")
    ap.add_argument("--gen-steps", type=int, default=250000)
    ap.add_argument("--gen-tol", type=float, default=1e-6)
    ap.add_argument("--eval-steps", type=int, default=2000000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--warmup", type=int, default=1000, help="iterations of linear learning-rate warm-up")
    ap.add_argument("--clip", type=float, default=2.0,
                    help="bound each step's gradient norm by this times the running average norm (0: off)")
    ap.add_argument("--dt", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=2019)
    ap.add_argument("--phase-seed", type=int, default=13,
                    help="seed of the random phase R(x, y) of Eq. (fun), shared by every instance "
                         "(13 as in the paper's programs); -1 draws one per instance")
    ap.add_argument("--weights", default=None, help="load weights (npz) and skip generate/train")
    ap.add_argument("--save-weights", default=None)
    ap.add_argument("--out", default=None, help="JSON summary path")
    ap.add_argument("--plain", action="store_true",
                    help="also run every evaluation instance alone from Eq. (fun)")
    ap.add_argument("--no-eval", action="store_true", help="generate and train only")
    ap.add_argument("--eval-3d", type=int, default=0,
                    help="with --weights: evaluate this many 3D instances (product start) instead")
    ap.add_argument("--lam", type=float, default=100.0, help="3D: trap frequency in z")
    ap.add_argument("--nz", type=int, default=16, help="3D: stored z points")
    ap.add_argument("--hz", type=float, default=0.05, help="3D: z spacing")
    a = ap.parse_args(argv)
    import torch

    def log(msg):
        print(msg, flush=True)

    res = {}
    if a.weights:
        params = load_params(a.weights)
    else:
        plist = draw(a.train, a.seed)
        seeds = [a.seed * 10 + k if a.phase_seed < 0 else a.phase_seed for k in range(a.train)]
        t0 = time.perf_counter()
        states, recs = generate(plist, seeds, dt=a.dt, max_steps=a.gen_steps, tol=a.gen_tol, log=log)
        res["generate_s"] = round(time.perf_counter() - t0, 1)
        res["generate_reached_tol"] = int(sum(1 for r in recs if r["steps"] > 0))
        X = _bf16_device(torch, features(plist))
        T = torch.tensor(make_targets(plist, states, a.dt), device="cuda")
        del states
        net = nn.UNet(a.batch, N_GRID, N_GRID, chans=CHANS, bott=BOTT, seed=a.seed)
        t0 = time.perf_counter()
        hist = train(net, X, T, a.epochs, lr=a.lr, seed=a.seed, log=log, warmup=a.warmup, clip=a.clip)
        torch.cuda.synchronize()
        res["train_s"] = round(time.perf_counter() - t0, 1)
        res["loss_history"] = [round(v, 5) for v in hist]
        params = net.params_numpy()
        if a.save_weights:
            save_params(a.save_weights, params)
        del X, T, net
    if a.no_eval:
        if a.out:
            with open(a.out, "w") as f:
                json.dump(res, f, indent=1)
        return
    if a.eval_3d:
        pl3 = draw(a.eval_3d, a.seed + 2)
        sd3 = [a.seed * 10 + 6000000 + k if a.phase_seed < 0 else a.phase_seed for k in range(a.eval_3d)]
        res["evaluate_3d"] = evaluate_3d(params, pl3, sd3, lam=a.lam, nz=a.nz, hz=a.hz, dt=a.dt,
                                         max_steps=a.eval_steps, log=log)
        log(json.dumps({k: v for k, v in res["evaluate_3d"].items() if k != "rows"}))
        if a.out:
            with open(a.out, "w") as f:
                json.dump(res, f, indent=1)
        return
    ev_plist = draw(a.eval, a.seed + 1)
    ev_seeds = [a.seed * 10 + 5000000 + k if a.phase_seed < 0 else a.phase_seed for k in range(a.eval)]
    res["evaluate"] = evaluate(params, ev_plist, ev_seeds, dt=a.dt, max_steps=a.eval_steps, plain=a.plain,
                               log=log)
    summary = {k: v for k, v in res["evaluate"].items() if k != "rows"}
    log(json.dumps(summary))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
