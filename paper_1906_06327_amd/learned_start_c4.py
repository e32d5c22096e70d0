"""Learned initial state at the scope of the batched sweep: a 256 x 256
network over the parameter ranges of the 64-instance batch, seeding
instances on their own grids.

The paper shortens imaginary-time runs by starting from a better state than
the one-vortex random-phase state of Eq. (fun) (Sec. 3, Fig. 3).  Here the
U-Net of nn.py proposes that state:

1. generate: parameter draws of the batched workload (Omega ~ U[0.5, 0.95],
   g ~ logU[100, 3000], nu ~ U[1.0, 1.2]; parameter seeds 1000..1031, 64
   draws each), each run by the batched solver from Eq. (fun) on the
   network's frame, a 256 x 256 grid spanning 2 x BOX Thomas-Fermi radii R,
   so that grid coordinates x / (BOX R) are the same for every instance and
   every instance starts from the same random phase field (phase seed 13):
   the lattice is then a function of (Omega, g, nu).  (Runs on the
   instances' own grids, whose sizes are drawn among the admissible ones,
   start from unrelated phase fields: their lattices are not a function of
   the parameters, and a network fitted to them learns only the density
   envelope.);
2. targets: the frame states.  Where the trap leaves the lattice orientation
   free (nu < NU_ISO: the two trap frequencies within 5 %), the target is
   rotated to a canonical orientation: the dominant angular order k of its
   density (the largest |M_k| / M_0, k = 2..8, sscn_angular_moments) put at
   phase 0.  Each target comes with its images under the symmetries of the
   rotating problem (rotation by pi, and each axis reflection with complex
   conjugation); the loss takes the nearest;
3. train: Adam on the phase-aligned loss, forward and backward on the bf16
   matrix-core kernels of include/sscn_nn.h;
4. propose: the network's output for an instance, resampled from the frame
   onto the instance's grid, walls zeroed and normalised;
5. evaluate: 64 held-out draws (parameter seed 4242) on their own grids,
   complex128, Delta = 1e-3, to |mu_n - mu_{n-1}| < 1e-8 at two consecutive
   checks 0.1 time units apart with an unchanged vortex count, in four arms:
   the plain method (each instance alone from Eq. (fun)), the learned start
   alone (each instance alone from its proposal), Eq. (fun) batched and the
   learned start batched.  The learned arms include inference and
   resampling in their wall time.

Generation runs complex64 sweeps (FP64 reductions) at Delta = 2e-3 for a
fixed imaginary time of 300 (150 000 steps), by which the lattices have
formed: the targets only need to be close to the converged lattice, since
the evaluation relaxes every proposal to 1e-8 in complex128 anyway.  (A
tolerance on the change of mu stops many instances during the transient,
long before the lattice has formed.)
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import Batch, angular_moments, resample
from . import nn
from .learned_start import _bf16_device, load_params, phase_distance, save_params, train

N_NET = 256
BOX = 1.35
CHANS = (32, 64, 128, 256, 256)
BOTT = 256
RANGES = dict(omega=(0.5, 0.95), g=(100.0, 3000.0), nu=(1.0, 1.2))
NU_ISO = 1.05
TRAIN_SEEDS = tuple(range(1000, 1032))
EVAL_SEED = 4242
PHASE_SEED = 13
GEN_DT, GEN_STEPS = 2e-3, 150000


def tf_radius(omega, g, nu):
    """Long Thomas-Fermi radius of the rotating 2D condensate: with
    a = 1 - Omega^2, b = nu^2 - Omega^2, mu = sqrt(g sqrt(a b) / pi) and
    R = sqrt(2 mu / a)."""
    a = 1.0 - omega * omega
    b = nu * nu - omega * omega
    mu = math.sqrt(g * math.sqrt(a * b) / math.pi)
    return math.sqrt(2.0 * mu / a)


def frame_h(c):
    """Spacing of the network frame of instance c: 2 BOX R / N_NET."""
    return 2.0 * BOX * tf_radius(c["omega"], c["g"], c["nu"]) / N_NET


def draws(seed, m=64):
    """m instances of the batched workload for parameter seed `seed` (grid
    side per instance from {128, ..., 512} at h = 0.1, Delta = 1e-3,
    complex128, phase seed 13 + n for the plain start)."""
    import workloads as W
    return W.batch_instances(n=m, seed=seed)


def features(cfgs, n=N_NET):
    """Network input (B, n, n, 16) fp32: x / (BOX R), y / (BOX R) on the
    frame, and Omega, log g, nu centred and scaled over their ranges;
    channels 5..15 zero."""
    ax = (np.arange(n) - n / 2) * 2.0 / n
    X, Y = np.meshgrid(ax, ax)
    om0, oms = 0.5 * sum(RANGES["omega"]), 0.5 * (RANGES["omega"][1] - RANGES["omega"][0])
    lg = [math.log(v) for v in RANGES["g"]]
    lg0, lgs = 0.5 * (lg[0] + lg[1]), 0.5 * (lg[1] - lg[0])
    nu0, nus = 0.5 * sum(RANGES["nu"]), 0.5 * (RANGES["nu"][1] - RANGES["nu"][0])
    f = np.zeros((len(cfgs), n, n, nn.IN_CH), np.float32)
    for k, c in enumerate(cfgs):
        f[k, ..., 0] = X
        f[k, ..., 1] = Y
        f[k, ..., 2] = (c["omega"] - om0) / oms
        f[k, ..., 3] = (math.log(c["g"]) - lg0) / lgs
        f[k, ..., 4] = (c["nu"] - nu0) / nus
    return f


def canonical_angle(m, nu):
    """Rotation (radians) that puts the dominant angular order k of a
    density at phase 0, from its moments m[k] = M_k (complex, k = 0..8);
    0 where the trap fixes the orientation (nu >= NU_ISO)."""
    if nu >= NU_ISO:
        return 0.0
    ratios = [abs(m[k]) / max(abs(m[0]), 1e-300) for k in range(2, len(m))]
    k = 2 + int(np.argmax(ratios))
    return float(np.angle(m[k]) / k)


def images(t):
    """(4, n, n, 2) fp32 images of a target (n, n, 2) on the centred square
    frame: itself, rotated by pi, conj(t(-x, y)), conj(t(x, -y)).  On the
    grid x_i = -n h / 2 + i h the reflection is the index map i -> (n - i)
    mod n (flip, then shift by one)."""
    import torch

    def refl(a, dim):
        return torch.roll(torch.flip(a, dims=(dim,)), shifts=1, dims=dim)

    def conj(a):
        return torch.stack((a[..., 0], -a[..., 1]), dim=-1)
    return torch.stack((t, refl(refl(t, 0), 1), conj(refl(t, 1)), conj(refl(t, 0))))


def _log_stderr(msg):
    print(msg, file=sys.stderr, flush=True)


def _run_chunks(b, max_steps, chk, tol, log, tag, chunk=50000):
    """sscn_batch_run in calls of `chunk` steps with a progress line after
    each; returns (steps per instance, seconds at which each converged)."""
    t0 = time.perf_counter()
    conv, when, done = [-1] * b.n, [None] * b.n, 0
    while done < max_steps and min(conv) < 0:
        m = min(chunk, max_steps - done)
        st = b.run(m, check_every=chk, tol=tol)
        done += m
        now = time.perf_counter() - t0
        for k, v in enumerate(st):
            if v >= 0 and conv[k] < 0:
                conv[k], when[k] = v, now
        log(f"[{tag}] {done} steps: {sum(1 for v in conv if v >= 0)}/{b.n} converged, {now:.1f} s")
    return conv, when


def frame_instance(c, dt=GEN_DT, precision=1):
    """Solver parameters of instance c on its network frame: N_NET points
    per axis at spacing frame_h(c)."""
    h = frame_h(c)
    return dict(dim=2, nx=N_NET, ny=N_NET, nz=1, hx=h, hy=h, hz=h, gamma=c["gamma"], nu=c["nu"], lam=1.0,
                g=c["g"], omega=c["omega"], dt=dt, mode=0, precision=precision)


def generate(param_seeds=TRAIN_SEEDS, log=_log_stderr):
    """Targets from the draws of every parameter seed, computed on the
    network frame itself (so that every instance starts from the same
    random phase field R(x / (BOX R), y / (BOX R)) of Eq. (fun), phase seed
    13, and its converged lattice is a function of (Omega, g, nu) alone):
    X (M, n, n, 16) bf16 and T (M, 4, n, n, 2) fp32 device tensors, and one
    record per instance."""
    import torch
    import workloads as W
    cfgs_all = []
    for sd in param_seeds:
        cfgs_all += draws(sd)
    M, n = len(cfgs_all), N_NET
    T = torch.empty((M, 4, n, n, 2), dtype=torch.float32, device="cuda")
    recs = []
    rot = torch.empty((n, n), dtype=torch.complex64, device="cuda")
    phase = W.phase_field(PHASE_SEED, n, n)
    m0 = 0
    for bi, sd in enumerate(param_seeds):
        cfgs = cfgs_all[m0:m0 + 64]
        gen = [frame_instance(c) for c in cfgs]
        b = Batch(gen)
        for k in range(len(gen)):
            b.init_state(k, 1, phase, 1.0)
        t0 = time.perf_counter()
        for done in range(0, GEN_STEPS, 25000):
            b.step(min(25000, GEN_STEPS - done))
            torch.cuda.synchronize()
            log(f"[generate {bi + 1}/{len(param_seeds)}] {min(done + 25000, GEN_STEPS)} steps, "
                f"{time.perf_counter() - t0:.1f} s")
        wall = time.perf_counter() - t0
        counts = [b.vortex_count(k) for k in range(len(cfgs))]
        for k, c in enumerate(cfgs):
            h = gen[k]["hx"]
            m = angular_moments(b.psi[k], (h, h), 8).cpu().numpy()
            ang = canonical_angle(m[:, 0] + 1j * m[:, 1], c["nu"])
            src = b.psi[k]
            if ang != 0.0:
                resample(src, (h, h), rot, (h, h), ang)
                src = rot
            nn.psi_to_f32(src, n * n, h * n / 4.0, T[m0 + k, 0])
            T[m0 + k] = images(T[m0 + k, 0])
            recs.append(dict(omega=c["omega"], g=c["g"], nu=c["nu"], h=h, vortices=counts[k], angle=round(ang, 6)))
        b.close()
        log(f"[generate] seed {sd}: {wall:.1f} s")
        m0 += 64
    X = _bf16_device(torch, features(cfgs_all))
    return X, T, recs


def propose(params, cfgs, dsts, log=None):
    """Write the learned start of every instance cfgs[k] into the device
    tensor dsts[k] (its grid, complex128): the network's output on the
    frame, resampled onto the instance's grid.  The caller zeroes the walls
    and normalises (set_state_device)."""
    import torch
    n = N_NET
    net = nn.UNet(len(cfgs), n, n, chans=CHANS, bott=BOTT, params=params)
    out = net.forward(_bf16_device(torch, features(cfgs)))
    frame = torch.empty((n, n), dtype=torch.complex128, device="cuda")
    for k, c in enumerate(cfgs):
        h = frame_h(c)
        nn.f32_to_psi(out[k], nn.OUT_CH, n * n, 1.0, frame)
        resample(frame, (h, h), dsts[k], (c["hx"], c["hy"]), 0.0)
    del net


def _single_arm(params, cfgs, max_steps, tol, learned, log, tag):
    """Every instance alone (a batch of one: the same kernels and criterion
    as the batched arm), from Eq. (fun) or from its learned start; returns
    per-instance rows and the total wall time (inference included)."""
    import torch
    import workloads as W
    chk = max(2, int(round(0.1 / cfgs[0]["dt"])))
    rows = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    starts = None
    t_inf = 0.0
    if learned:
        starts = [torch.empty((c["ny"], c["nx"]), dtype=torch.complex128, device="cuda") for c in cfgs]
        propose(params, cfgs, starts)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t_all
    for k, c in enumerate(cfgs):
        t0 = time.perf_counter()
        b = Batch([c])
        if learned:
            b.psi[0].copy_(starts[k])
            b.set_state_device(0)  # walls zeroed, normalised
        else:
            b.init_state(0, 1, W.phase_field(c["seed"], c["ny"], c["nx"]), 1.0)
        st = b.run(max_steps, check_every=chk, tol=tol)[0]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rows.append(dict(steps=st, wall_s=round(wall, 4), vortices=b.vortex_count(0), mu=b.observables()[0]["mu"]))
        b.close()
        log(f"[{tag}] {k + 1}/{len(cfgs)} n={c['nx']}: {st} steps, {wall:.2f} s, {rows[-1]['vortices']} vortices")
    torch.cuda.synchronize()
    return rows, time.perf_counter() - t_all, t_inf


def _batch_arm(params, cfgs, max_steps, tol, learned, log, tag):
    """All instances in one batch from Eq. (fun) or from the learned starts."""
    import torch
    import workloads as W
    chk = max(2, int(round(0.1 / cfgs[0]["dt"])))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = Batch(cfgs)
    t_inf = 0.0
    if learned:
        propose(params, cfgs, b.psi)
        for k in range(len(cfgs)):
            b.set_state_device(k)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
    else:
        for k, c in enumerate(cfgs):
            b.init_state(k, 1, W.phase_field(c["seed"], c["ny"], c["nx"]), 1.0)
    starts = [b.get_state(k) for k in range(len(cfgs))]
    steps, when = _run_chunks(b, max_steps, chk, tol, log, tag)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    obs = b.observables()
    rows = [dict(steps=steps[k], seconds=None if when[k] is None else round(when[k], 3),
                 vortices=b.vortex_count(k), mu=obs[k]["mu"]) for k in range(len(cfgs))]
    finals = [b.get_state(k) for k in range(len(cfgs))]
    b.close()
    return rows, wall, t_inf, starts, finals


def evaluate(params, arms=("batched", "single"), seed=EVAL_SEED, max_steps=2000000, tol=1e-8,
             log=_log_stderr):
    """The four arms on the held-out draws of `seed` (see the module
    docstring); `arms` selects among "batched" (both batched arms),
    "single" (both one-at-a-time arms), "plain" and "learned_alone"."""
    cfgs = draws(seed)
    res = dict(seed=seed, instances=len(cfgs), tol=tol, max_steps=max_steps, dt=cfgs[0]["dt"],
               grid_sides=[c["nx"] for c in cfgs],
               params=[dict(omega=round(c["omega"], 5), g=round(c["g"], 3), nu=round(c["nu"], 5)) for c in cfgs])
    if "batched" in arms:
        r0, w0, _, s0, f0 = _batch_arm(params, cfgs, max_steps, tol, False, log, "batched Eq. (fun)")
        r1, w1, i1, s1, f1 = _batch_arm(params, cfgs, max_steps, tol, True, log, "batched learned")
        res["batched_one_vortex"] = dict(wall_s=round(w0, 3), rows=r0)
        res["batched_learned"] = dict(wall_s=round(w1, 3), inference_and_resampling_s=round(i1, 3), rows=r1)
        # distance of each start from the lattice the Eq. (fun) run converged to
        res["distance_to_converged"] = dict(
            one_vortex=[round(phase_distance(s0[k], f0[k]), 5) for k in range(len(cfgs))],
            learned=[round(phase_distance(s1[k], f0[k]), 5) for k in range(len(cfgs))])
    if "single" in arms or "plain" in arms:
        r2, w2, _ = _single_arm(params, cfgs, max_steps, tol, False, log, "plain")
        res["plain"] = dict(wall_s=round(w2, 3), rows=r2)
    if "single" in arms or "learned_alone" in arms:
        r3, w3, i3 = _single_arm(params, cfgs, max_steps, tol, True, log, "learned alone")
        res["learned_alone"] = dict(wall_s=round(w3, 3), inference_and_resampling_s=round(i3, 3), rows=r3)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description="Learned initial state over the batched workload's ranges.")
    ap.add_argument("--seeds", type=int, default=len(TRAIN_SEEDS), help="parameter seeds of training data (64 each)")
    ap.add_argument("--epochs", type=int, default=25)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--clip", type=float, default=2.0)
    ap.add_argument("--weights", default=None, help="load weights (npz) and skip generation and training")
    ap.add_argument("--save-weights", default=None)
    ap.add_argument("--evaluate", default="", help="comma list of arms: batched, single, plain, learned_alone")
    ap.add_argument("--eval-steps", type=int, default=2000000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    import torch
    res = {}
    if a.weights:
        params = load_params(a.weights)
    else:
        t0 = time.perf_counter()
        X, T, recs = generate(TRAIN_SEEDS[:a.seeds])
        torch.cuda.synchronize()
        res["generate_s"] = round(time.perf_counter() - t0, 1)
        res["generate"] = recs
        net = nn.UNet(a.batch, N_NET, N_NET, chans=CHANS, bott=BOTT, seed=2019)
        t0 = time.perf_counter()
        hist = train(net, X, T, a.epochs, lr=a.lr, seed=2019, log=_log_stderr, log_every=100, warmup=a.warmup,
                     clip=a.clip)
        torch.cuda.synchronize()
        res["train_s"] = round(time.perf_counter() - t0, 1)
        res["loss_history"] = [round(v, 5) for v in hist]
        params = net.params_numpy()
        if a.save_weights:
            save_params(a.save_weights, params)
        del X, T, net
        torch.cuda.empty_cache()
    if a.evaluate:
        res["evaluate"] = evaluate(params, arms=tuple(a.evaluate.split(",")), max_steps=a.eval_steps)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps({k: v for k, v in res.items() if k not in ("generate", "evaluate")}), flush=True)


if __name__ == "__main__":
    main()
