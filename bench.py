"""Benchmark of the SSCN hot path on one MI355X.

Workload (default, the headline): the batched 2D imaginary-time sweep of 64
instances of uneven size and parameters (parameter seed 2019): grid sides
from {128, 192, 256, 384, 512} at h = 0.1 (each side holding 2 x 1.4
Thomas-Fermi radii), Omega ~ U[0.5, 0.95], g ~ logU[100, 3000],
nu ~ U[1.0, 1.2], gamma = 1, dt = 1e-3, complex128 arithmetic, renormalised
every step, each instance starting from the one-vortex random-phase state of
Eq. (fun) (phase seed 13 + n).  One step advances every instance by one full
SSCN step (H1 + x-sweep + y-sweep + FP64 norm; the rescale is folded into
the next step).  `value` = grid-point updates per second, sum over the
instances of their points times --steps, over the wall time of exactly
--steps timed steps; the inputs are resident on the GPU and the steps are
replayed from HIP graphs captured before the timed region.  Before the
--warmup steps, untimed chunks of 50 steps run until two consecutive chunks
agree in time to 1 % (at most 2 s), so that a timed region of a few
milliseconds does not measure the clock ramp of a GPU that was idle.

Also reported on the same JSON line:
  roofline      the dominant kernel of the batched step: algorithmic bytes
                per launch (one read and one write of every instance's state
                per sweep: 2 x 16 B per point) / its average duration,
                measured with HIP events (without system-scope fences)
                around every kernel of consecutive steps on the stream it
                runs on, against 8 TB/s HBM; traffic =
                counter bytes per launch from the committed rocprofv3 summary
                (null when the kernel sources differ from the ones profiled);
  variants      the 512^2 workload (complex128 and complex64, imaginary and
                real time), the 3D 256 x 256 x 64 workload (complex64 and
                complex128), each followed by real-time steps with norm and
                energy drift; a batch of 8 3D instances (complex64 and
                complex128); the learned start's network (forward pass and
                training iteration at 256^2, batch 16, against the bf16
                matrix-core peak);
  converge      time to converged lattices: the 128^2 workload (complex128;
                complex64 then complex128) and, per instance, the 64-instance
                batch (mu changing by < 1e-8 over 0.1 time units at two
                consecutive checks with an unchanged vortex count);
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the headline
                workload (consecutive steps of each instance in turn) on the
                host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ("paper_1906_06327_amd/csrc/sscn_device.hpp", "paper_1906_06327_amd/csrc/sscn_host.hpp",
                  "paper_1906_06327_amd/csrc/sscn_kernels.hip", "paper_1906_06327_amd/csrc/sscn_lib.hip")
HEADLINE = ("2D rotating GP, 64 instances (parameter seed 2019) with grid sides from "
            "{128,192,256,384,512} at h=0.1, Omega~U[0.5,0.95], g~logU[100,3000], nu~U[1.0,1.2], "
            "gamma=1, dt=1e-3, imaginary time, renormalised each step, one batched launch per kernel")


def source_hash():
    """sha256 over the solver kernel sources, in KERNEL_SOURCES order."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(key):
    """HBM bytes per launch of a kernel from its committed counter summary
    (profiles/traffic_<key>.md: FETCH_SIZE and WRITE_SIZE passes scaled by
    the plain-copy calibration), or None when the summary is missing or was
    taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{key}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip(" -*`")] = v.strip(" `\n")
    if vals.get("source_sha256") != source_hash():
        return None
    try:
        return int(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--precision", choices=("c128", "c64"), default="c128")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip variants and convergence runs")
    ap.add_argument("--no-batch-converge", action="store_true",
                    help="skip the 64-instance convergence run (the longest extra)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--profile-sample", action="store_true",
                    help="run a short fixed sample for hardware-counter passes and exit: a "
                         "256 MiB device copy (counter calibration), 20 steps of the 64-instance "
                         "complex128 batch, 50 steps of the 512^2 complex128 workload, 20 steps "
                         "of the 3D complex64 workload")
    ap.add_argument("--profile-network", action="store_true",
                    help="run a short fixed sample of the learned start's network for a kernel trace and "
                         "exit: 3 forward passes and 2 training iterations at 256^2, batch 16")
    return ap.parse_args()


def sync(torch):
    torch.cuda.synchronize()


def make_batch(P, cfgs):
    b = P.Batch(cfgs)
    for k, c in enumerate(cfgs):
        b.init_state(k, c.get("kind", 1), W.phase_field(c["seed"], c["ny"], c["nx"]), c.get("d_xy", 1.0))
    return b


def batch_cfgs(precision):
    return [dict(c, precision=precision) for c in W.batch_instances()]


def profile_sample(P, torch):
    n = 256 * 1024 * 1024 // 16
    a = torch.ones(n, dtype=torch.complex128, device="cuda")
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    sync(torch)
    print("profile-sample: copy 256 MiB x3 done", flush=True)
    del a, c
    # the plan and x-sweep lines-per-block option the headline's autotuner
    # picks on this workload (under a counter-collecting profiler the
    # autotuner's own timings are distorted)
    os.environ["SSCN_BATCH_XLINES"] = "1"
    b = make_batch(P, batch_cfgs(0))
    del os.environ["SSCN_BATCH_XLINES"]
    b.set_plan(P.PLAN_SWEEPS)
    b.prepare_steps(20)
    b.step(20)
    sync(torch)
    print(f"profile-sample: 64-instance batch, 20 steps, plan {b.info()['plan']}", flush=True)
    b.close()
    for cfg, k in ((W.CONFIGS["c2"], 50), (W.CONFIGS["c3"], 20)):
        s = P.Solver(W.solver_params(cfg))
        s.init_state(1, W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"]), 1.0, cfg.get("d_z", 0.0))
        s.step(k)
        sync(torch)
        print(f"profile-sample: {cfg['nx']}x{cfg['ny']}x{cfg['nz']} {k} steps, "
              f"plan {s.solver_info()['plan']}", flush=True)
        s.close()


def settle(obj, torch, chunk=50, tol=0.01, max_s=2.0):
    """Untimed steps in chunks until two consecutive chunks take the same time
    to within tol (HIP events on the current stream, which the object
    launches on), at most max_s seconds: a GPU that has been idle runs its
    first milliseconds of work at lower clocks, which a timed region of a few
    milliseconds would otherwise measure.  Returns the chunks' ms per step."""
    obj.prepare_steps(chunk)
    times, t_end = [], time.perf_counter() + max_s
    while time.perf_counter() < t_end:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        obj.step(chunk)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / chunk)
        if len(times) >= 3 and abs(times[-1] - times[-2]) <= tol * times[-1]:
            break
    return times


def timed_batch(P, torch, cfgs, steps, warmup, info=None):
    """The headline: settle the clocks (settle), warm up, capture the graphs
    of a `steps`-step call, then time exactly `steps` steps (wall clock
    between two synchronisations, and HIP events on the batch's stream around
    the same region).  info (a dict) receives the settling chunks."""
    b = make_batch(P, cfgs)
    st = settle(b, torch)  # the batch launches on torch's current stream
    if info is not None:
        info["settle_ms_per_step"] = [round(t, 5) for t in st]
    b.prepare_steps(warmup)
    b.step(warmup)
    b.prepare_steps(steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sync(torch)
    t0 = time.perf_counter()
    e0.record()
    b.step(steps)
    e1.record()
    sync(torch)
    dt = time.perf_counter() - t0
    return b, dt, e0.elapsed_time(e1) / steps


def batch_roofline(b, cfgs, nprof=20):
    """Average duration of each kernel of the batched step, from HIP events
    recorded around every kernel of nprof consecutive steps on the batch's
    stream (sscn_batch_profile_step), and the algorithmic bandwidth of the
    dominant one: one read and one write of every instance's state per sweep
    (2 c bytes per point, c = complex size), i.e. 2 c sum(P) per sweep kernel
    and 2 x 2 c sum(P) for the fused step (both sweeps in one launch)."""
    prof = b.profile_step(nprof)
    esize = 16 if cfgs[0]["precision"] == 0 else 8
    pts = sum(c["nx"] * c["ny"] for c in cfgs)
    prec = "c128" if esize == 16 else "c64"
    if "fused" in prof:
        names, per_launch, label = ("fused",), 2 * 2 * esize * pts, "batched fused 2D step (H1 + x + y)"
        keys = {"fused": f"batch64_fused2d_{prec}"}
    else:
        names, per_launch = ("x", "y"), 2 * esize * pts
        keys = {"x": f"batch64_xsweep_{prec}", "y": f"batch64_ysweep_{prec}"}
    dom = max(names, key=lambda k: prof[k])
    if "fused" not in prof:
        label = {"x": "batched x-sweep (H1 + rescale + x-CN), k_batch_xsweep",
                 "y": "batched y-sweep (y-CN + norm partials), k_batch_ysweep"}[dom]
    gbs = per_launch / (prof[dom] * 1e-3) / 1e9
    traffic = measured_traffic(keys[dom])
    out = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic,
           "traffic_unit": "bytes per launch (counters)",
           "traffic_over_algorithmic": round(traffic / per_launch, 3) if traffic else None,
           "kernel": label, "bytes_per_launch": per_launch,
           "kernel_ms": {k: round(v, 6) for k, v in prof.items()},
           "timing": f"HIP events around every kernel of {nprof} consecutive steps"}
    others = {}
    for k in names:
        if k != dom:
            g = per_launch / (prof[k] * 1e-3) / 1e9
            others[k] = {"achieved": round(g, 1), "frac": round(g / PEAK_HBM_GBS, 4),
                         "traffic": measured_traffic(keys[k])}
    if others:
        out["other_kernels"] = others
    return out


def timed_steps(P, torch, cfg, steps, warmup, mode=0):
    """Warm up, capture the graphs of a `steps`-step call, then time exactly
    `steps` steps: wall clock between two synchronisations, and HIP events
    recorded on the solver's stream (the current torch stream, which the
    solver launches on) around the same region.  Returns (solver, wall
    seconds, event milliseconds per step)."""
    s = P.Solver(W.solver_params(cfg, mode=mode), stream=torch.cuda.current_stream())
    ph = W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"])
    s.init_state(cfg.get("kind", 1), ph, cfg.get("d_xy", 1.0), cfg.get("d_z", 0.0))
    s.prepare_steps(warmup)
    s.step(warmup)
    s.prepare_steps(steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sync(torch)
    t0 = time.perf_counter()
    e0.record()
    s.step(steps)
    e1.record()
    sync(torch)
    dt = time.perf_counter() - t0
    return s, dt, e0.elapsed_time(e1) / steps


def batch3d_variant(P, torch, precision, steps=200, warmup=20):
    """The batched 3D sweep (workloads.batch3d_instances: 8 instances of the
    3D workload's trap with different rotations, couplings and in-plane
    sides): updates/s over `steps` graph-replayed steps and the average
    duration of its x-, y- and z-sweep kernels (HIP events around every
    kernel of 10 steps), with their algorithmic bandwidth (2 c bytes per
    point per sweep)."""
    cfgs = [dict(c, precision=precision) for c in W.batch3d_instances()]
    pts = sum(c["nx"] * c["ny"] * c["nz"] for c in cfgs)
    b, dt, _ = timed_batch(P, torch, cfgs, steps, warmup)
    prof = b.profile_step(10)
    xopt = b.info()["x_lines_option"]
    b.close()
    esize = 16 if precision == 0 else 8
    per = 2 * esize * pts
    return {"instances": len(cfgs), "points": pts, "grid_sides": sorted({c["nx"] for c in cfgs}),
            "nz": cfgs[0]["nz"], "x_lines_option": xopt, "updates_per_s": round(pts * steps / dt, 1),
            "ms_per_step": round(dt / steps * 1e3, 6), "steps": steps,
            "kernel_ms": {k: round(v, 6) for k, v in prof.items()},
            "kernel_frac_of_8TBps": {k: round(per / (prof[k] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)
                                     for k in ("x", "y", "z")}}


def real_time_phase(P, torch, s, steps):
    """From the solver's current imaginary-time state, `steps` real-time
    steps (same grid and precision): wall time and the drift of the norm
    and of the full energy functional, which real time conserves up to the
    splitting error."""
    o0 = s.observables()
    s.set_mode(P.SSCN_REAL)
    s.prepare_steps(steps)
    sync(torch)
    t0 = time.perf_counter()
    s.step(steps)
    sync(torch)
    dt = time.perf_counter() - t0
    o1 = s.observables()
    return {"steps": steps, "ms_per_step_timed": round(dt / steps * 1e3, 6),
            "norm_drift": o1["norm"] - o0["norm"],
            "energy_full_rel_drift": (o1["energy_full"] - o0["energy_full"]) / abs(o0["energy_full"])}


def kernel_roofline(s, cfg, step_ms, nlaunch=200):
    """Average duration of the dominant kernel of a single-instance step and
    its algorithmic bandwidth.  The fused 2D plan launches one kernel per
    step, so its duration is the event time of the timed region per step.
    The sweep plans launch one kernel per axis; each is timed over nlaunch
    back-to-back launches between two HIP events on the solver's stream
    (sscn_profile_kernel).  Algorithmic bytes: 2 c per point per axis sweep
    the kernel performs."""
    info = s.solver_info()
    plan = info["plan"]
    dim = cfg["dim"]
    pts = cfg["nx"] * cfg["ny"] * (cfg["nz"] if dim == 3 else 1)
    esize = 16 if cfg.get("precision", 0) == 0 else 8
    if plan == 2:
        names, per_launch = ("fused",), 2 * dim * esize * pts
        ms = {"fused": step_ms}
    else:
        names, per_launch = ("x", "y", "z")[:dim], 2 * esize * pts
        ms = {k: s.profile_kernel(w, nlaunch) for w, k in enumerate(names)}
    dom = max(names, key=lambda k: ms[k])
    gbs = per_launch / (ms[dom] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4),
            "kernel": "fused 2D step (H1 + x + y)" if plan == 2 else f"{dom}-sweep",
            "plan": {1: "sweeps", 2: "fused"}.get(plan, plan),
            "tile": info["fused_tile"] if plan == 2 else None, "bytes_per_launch": per_launch,
            "kernel_ms": {k: round(v, 6) for k, v in ms.items()},
            "timing": "events around the timed steps" if plan == 2 else "events around back-to-back launches"}


def single_variant(P, torch, cfg, steps, warmup, real_steps=0, mode=0):
    s, dt, sm = timed_steps(P, torch, cfg, steps, warmup, mode=mode)
    pts = cfg["nx"] * cfg["ny"] * (cfg["nz"] if cfg["dim"] == 3 else 1)
    out = {"updates_per_s": round(pts * steps / dt, 1), "ms_per_step": round(dt / steps * 1e3, 6),
           "steps": steps, "roofline": kernel_roofline(s, cfg, sm)}
    if real_steps:
        out["then_real_time"] = real_time_phase(P, torch, s, real_steps)
    s.close()
    return out


def converge_run(P, torch, cfg, precision, max_steps=3000000):
    """Imaginary time from Eq. (fun) to |mu_n - mu_{n-1}| < 1e-8 at two
    consecutive checks 0.1 time units apart with the vortex count unchanged
    (sscn_converge; complex64 bulk switches to complex128 at its plateau)."""
    s = P.Solver(W.solver_params(cfg, precision=precision))
    ph = W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"])
    chk = max(1, int(round(0.1 / cfg["dt"])))
    sync(torch)
    t0 = time.perf_counter()
    s.init_state(1, ph, 1.0)
    steps, ok = s.converge(max_steps, check_every=chk, tol=1e-8, switch_tol=3e-7)
    sync(torch)
    wall = time.perf_counter() - t0
    ob = s.observables()
    out = {"precision": "c128" if precision == 0 else "c64 bulk -> c128", "steps": steps,
           "converged": ok, "wall_s": round(wall, 3), "mu": ob["mu"], "energy": ob["energy"],
           "vortices": s.vortex_count(), "fp32_steps": s.switch_step if precision == 1 else 0}
    s.close()
    return out


def batch_converge(P, torch, cfgs, max_steps=2000000, chunk=20000):
    """The 64 instances from Eq. (fun) to the convergence criterion, all in
    one batch (sscn_batch_run, checks every 0.1 time units on the device,
    converged instances leave the batch).  The run is driven in calls of
    `chunk` steps, so that each instance's convergence is also timed (to the
    end of the call in which it converged)."""
    chk = max(2, int(round(0.1 / cfgs[0]["dt"])))
    sync(torch)
    t0 = time.perf_counter()
    b = make_batch(P, cfgs)
    conv = [-1] * len(cfgs)
    when = [None] * len(cfgs)
    done = 0
    while done < max_steps and min(conv) < 0:
        st = b.run(min(chunk, max_steps - done), check_every=chk, tol=1e-8)
        done += min(chunk, max_steps - done)
        now = time.perf_counter() - t0
        for k, v in enumerate(st):
            if v >= 0 and conv[k] < 0:
                conv[k], when[k] = v, now
        print(f"[bench] batch convergence: {done} steps, {sum(1 for v in conv if v >= 0)}/{len(conv)} "
              f"converged, {now:.1f} s", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    counts = [b.vortex_count(k) for k in range(len(cfgs))]
    obs = b.observables()
    b.close()
    ok = [k for k in range(len(cfgs)) if conv[k] >= 0]
    pts = [c["nx"] * c["ny"] for c in cfgs]
    st = sorted(conv[k] for k in ok)
    tm = sorted(when[k] for k in ok)
    return {"instances": len(cfgs), "converged": len(ok), "wall_s": round(wall, 3),
            "max_steps": max_steps, "check_every": chk,
            "steps_min_median_max": [st[0], st[len(st) // 2], st[-1]] if st else None,
            "seconds_min_median_max": [round(tm[0], 3), round(tm[len(tm) // 2], 3), round(tm[-1], 3)] if tm else None,
            "per_instance": [{"n": c["nx"], "omega": round(c["omega"], 4), "g": round(c["g"], 2),
                              "nu": round(c["nu"], 4), "steps": conv[k],
                              "seconds": None if when[k] is None else round(when[k], 3),
                              "vortices": counts[k], "mu": obs[k]["mu"]} for k, c in enumerate(cfgs)],
            "updates": int(sum(pts[k] * (conv[k] if conv[k] >= 0 else done) for k in range(len(cfgs))))}


def _omp_threads(n):
    """Set the OpenMP thread count of this process's runtime (the oracle's
    library shares it); returns False where libgomp cannot be loaded."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def oracle_rate(cfg, seconds, chunk=25):
    """Updates/s of the FP64 oracle over consecutive steps of cfg from its
    initial state, for about `seconds` of host time."""
    import oracle as O
    p = O.make_params(**W.solver_params(cfg))
    ph = W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"])
    psi = O.init_state(p, 1, ph, 1.0)
    psi = O.step(p, psi, 2)  # warm-up
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        psi = O.step(p, psi, chunk)
        steps += chunk
    dt = time.perf_counter() - t0
    return cfg["nx"] * cfg["ny"] * steps / dt, steps, dt


def oracle_batch_rate(cfgs, seconds, steps_each=2):
    """Updates/s of the FP64 oracle on the batch workload: rounds over the
    instances, each advancing its own state by `steps_each` consecutive steps
    (timed; the initial states are not), until about `seconds` of stepping.
    Returns (rate, rounds, instances stepped in the last round, seconds)."""
    import oracle as O
    ps = [O.make_params(**W.solver_params(c)) for c in cfgs]
    states = [None] * len(cfgs)
    upd, spent, rounds, inst = 0, 0.0, 0, 0
    while spent < seconds:
        rounds += 1
        for k, c in enumerate(cfgs):
            if states[k] is None:
                states[k] = O.init_state(ps[k], 1, W.phase_field(c["seed"], c["ny"], c["nx"]), 1.0)
            t0 = time.perf_counter()
            states[k] = O.step(ps[k], states[k], steps_each)
            spent += time.perf_counter() - t0
            upd += c["nx"] * c["ny"] * steps_each
            inst = k + 1
            if spent >= seconds:
                break
    return upd / spent, rounds, inst, spent


def cpu_baseline(cfgs, seconds):
    """The FP64 oracle as it stands on the host cores, on a bounded sample of
    the headline workload (rounds over the 64 instances, two consecutive
    steps of each per round)."""
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rate, rounds, inst, dt = oracle_batch_rate(cfgs, seconds)
    out = {"value": round(rate, 1), "unit": "updates/s", "cores": threads, "kind": "oracle",
           "sample": f"imaginary-time steps of the 64 batch instances (complex128), 2 consecutive steps of "
                     f"each instance per round, {rounds} round(s), the last ending at instance {inst}; "
                     f"{dt:.1f} s of stepping, OpenMP over lines with {threads} threads"}
    if _omp_threads(1):
        r1, rd1, i1, d1 = oracle_batch_rate(cfgs, seconds / 3)
        _omp_threads(threads)
        out["single_thread"] = {"value": round(r1, 1), "unit": "updates/s", "cores": 1,
                                "sample": f"the same, {rd1} round(s) ending at instance {i1} ({d1:.1f} s)"}
    return out


PEAK_BF16_TFLOPS = 2500.0


def conv_flops(net):
    """Multiply-add flops (2 per product) of the network's 3x3 convolutions
    in one forward pass of net.N samples."""
    return sum(2.0 * net.N * net.shapes[n][0] * net.shapes[n][1] * 9 * cin * cout for n, cin, cout, _ in net.specs)


def network_rate(P, torch, N=16, H=256, reps=10):
    """The learned start's network (6 levels, 32-64-128-256-256 channels and a
    256-channel bottleneck, 256 x 256 points, batch N): average time of a
    forward pass and of a training iteration (forward, loss, backward, Adam)
    over `reps` calls between HIP events, and their convolution flop rates
    against the dense bf16 matrix-core peak.  The backward pass does twice
    the forward's convolution flops (input and weight gradients)."""
    from paper_1906_06327_amd import nn
    net = nn.UNet(N, H, H, chans=(32, 64, 128, 256, 256), bott=256, seed=7)
    rng = np.random.default_rng(7)
    xf = rng.standard_normal((N, H, H, nn.IN_CH)).astype(np.float32)
    x = torch.tensor(xf, device="cuda").to(torch.bfloat16).view(torch.int16)
    tgt = torch.tensor(rng.standard_normal((N, H, H, 2)).astype(np.float32), device="cuda")
    fl = conv_flops(net)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        net.forward(x)
    sync(torch)
    e0.record()
    for _ in range(reps):
        net.forward(x)
    e1.record()
    sync(torch)
    fwd_ms = e0.elapsed_time(e1) / reps

    def train_iter():
        net.forward(x)
        net.loss_and_grad(tgt)
        net.backward(net.gacts["out"])
        net.adam_step(lr=1e-5)
    train_iter()
    sync(torch)
    t0 = time.perf_counter()
    for _ in range(reps):
        train_iter()
    sync(torch)
    it_ms = (time.perf_counter() - t0) / reps * 1e3
    fwd_tf = fl / (fwd_ms * 1e-3) / 1e12
    it_tf = 3 * fl / (it_ms * 1e-3) / 1e12
    return {"network": "U-Net, 6 levels, 32-64-128-256-256 + 256 bottleneck", "batch": N, "grid": [H, H],
            "conv_gflop_forward": round(fl / 1e9, 1), "forward_ms": round(fwd_ms, 3),
            "forward_tflops": round(fwd_tf, 1), "forward_frac_bf16_peak": round(fwd_tf / PEAK_BF16_TFLOPS, 4),
            "train_iteration_ms": round(it_ms, 3), "train_tflops": round(it_tf, 1),
            "train_frac_bf16_peak": round(it_tf / PEAK_BF16_TFLOPS, 4), "peak_tflops": PEAK_BF16_TFLOPS,
            "timing": f"forward: HIP events over {reps} passes; training: wall clock over {reps} iterations "
                      f"(the loss reads its value back to the host each iteration)"}


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """GB/s of a plain device-to-device copy (read + write counted), timed
    with HIP events: the achievable HBM bandwidth the kernels are also
    compared with."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    sync(torch)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    sync(torch)
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus > 1 or world > 1:
        print(f"bench.py measures one GPU only: this build runs on a single GPU and has no "
              f"multi-GPU path (asked for --gpus {a.gpus}, WORLD_SIZE {world}).", flush=True)
        sys.exit(2)
    import torch
    import paper_1906_06327_amd as P
    P.lib()
    torch.cuda.set_device(0)
    if a.profile_sample:
        profile_sample(P, torch)
        return
    if a.profile_network:
        r = network_rate(P, torch, reps=2)
        print(f"profile-network: forward {r['forward_ms']} ms ({r['forward_tflops']} TFLOP/s), training "
              f"iteration {r['train_iteration_ms']} ms", flush=True)
        return

    prec = 0 if a.precision == "c128" else 1
    cfgs = batch_cfgs(prec)
    pts = sum(c["nx"] * c["ny"] for c in cfgs)
    sinfo = {}
    b, dt, step_ms = timed_batch(P, torch, cfgs, a.steps, a.warmup, info=sinfo)
    value = pts * a.steps / dt
    roof = batch_roofline(b, cfgs)
    info = b.info()
    b.close()
    roof["copy_GBps"] = round(copy_bandwidth(torch), 1)
    roof["frac_of_copy"] = round(roof["achieved"] / roof["copy_GBps"], 4)
    sizes = {}
    for c in cfgs:
        sizes[c["nx"]] = sizes.get(c["nx"], 0) + 1

    out = {
        "metric": "grid-point updates/s per SSCN step (% HBM roofline) + time-to-converged lattice",
        "value": round(value, 1), "unit": "updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(dt / a.steps * 1e3, 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32",
        "data": "synthetic (one-vortex random-phase initial states, phase seeds 13 + n)",
        "config": {"workload": HEADLINE, "instances": len(cfgs), "points": pts,
                   "grid_sides": {str(k): v for k, v in sorted(sizes.items())},
                   "precision": a.precision, "plan": {1: "batched sweeps", 2: "batched fused step"}.get(
                       info["plan"], info["plan"]), "window": info["window"],
                   "x_lines": {0: "most lines per block", 1: "lines per block capped at 40 KiB of LDS"}[
                       info["x_lines_option"]],
                   "x_lines_tune_ms_8_steps": [round(t, 4) for t in info["x_lines_tune_ms"]],
                   "step_ms_events": round(step_ms, 6), "parallelism": "single GPU"},
        "roofline": roof,
        "settle": {"steps_per_chunk": 50, "ms_per_step": sinfo["settle_ms_per_step"],
                   "note": "untimed chunks of steps before the warm-up, until two agree to 1 %"},
    }
    if not a.no_extras:
        variants = {}
        c2 = W.CONFIGS["c2"]
        variants["c2_512_complex128"] = single_variant(P, torch, c2, 5120, 256, real_steps=10240)
        variants["c2_512_complex64"] = single_variant(P, torch, dict(c2, precision=1), 5120, 256)
        variants["c2_512_real_time_complex128"] = single_variant(P, torch, c2, 5120, 256, mode=1)
        c3 = W.CONFIGS["c3"]
        variants["c3_3d_complex64"] = single_variant(P, torch, c3, 1024, 64, real_steps=1024)
        variants["c3_3d_complex128"] = single_variant(P, torch, dict(c3, precision=0), 512, 64, real_steps=512)
        variants["batch_3d_8_complex64"] = batch3d_variant(P, torch, 1)
        variants["batch_3d_8_complex128"] = batch3d_variant(P, torch, 0, steps=100)
        variants["learned_start_network"] = network_rate(P, torch)
        out["variants"] = variants
        c1 = W.CONFIGS["c1"]
        conv = {"workload": "2D 128x128 on [-6.4,6.4)^2, g=100, Omega=0.6, dt=1e-3, one-vortex "
                            "random-phase start (seed 13)",
                "criterion": "|dmu| < 1e-8 at two consecutive checks 0.1 time units apart, "
                             "vortex count unchanged"}
        conv["c128"] = converge_run(P, torch, c1, 0)
        conv["c64_then_c128"] = converge_run(P, torch, c1, 1)
        if not a.no_cpu:
            # the oracle on the same lattice: its measured rate times the
            # GPU run's step count (a full oracle run would take minutes)
            rate, steps, dto = oracle_rate(c1, 3.0)
            conv["c128"]["oracle_extrapolated_s"] = round(conv["c128"]["steps"] * c1["nx"] * c1["ny"] / rate, 1)
            conv["c128"]["oracle_sample"] = f"{steps} oracle steps in {dto:.1f} s on the host cores"
        if not a.no_batch_converge:
            conv["batch_64_complex128"] = batch_converge(P, torch, batch_cfgs(0))
        out["converge"] = conv
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfgs, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
