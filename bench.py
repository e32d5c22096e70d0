"""Benchmark of the SSCN hot path on one MI355X.

Workload (default): the 2D rotating-GP problem on a 512 x 512 grid on
[-12.8, 12.8)^2, gamma = 1, nu = 1.05, g = 1000, Omega = 0.9, dt = 5e-4,
imaginary time with renormalisation every step, complex128 arithmetic,
starting from the one-vortex random-phase state of Eq. (fun) (seed 13).
One step = H1 + x-sweep + y-sweep + FP64 norm (the rescale is folded into
the next step).  `value` = grid-point updates per second over exactly
--steps timed steps, inputs resident on the GPU.

Also reported on the same JSON line:
  roofline      the dominant sweep kernel: algorithmic bytes (one read and
                one write of the state) / its average duration measured with
                HIP events on the stream it runs on, against 8 TB/s HBM;
  variants      the same workload with complex64 sweeps, in real time from
                the start, and in real time from the timed run's state
                (10 000 steps, norm and energy drift); the 3D 256 x 256 x 64
                complex64 workload (then 1 000 real-time steps); the
                64-instance batch;
  converge      time to a converged lattice on the 128^2 workload (mu
                changing by < 1e-8 over 0.1 time units at two consecutive
                checks with an unchanged vortex count);
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the default
                workload, on the host cores (and on one thread).
The roofline object also carries the bandwidth of a plain 1 GiB device copy
(copy_GBps), the achievable figure next to the 8 TB/s specification, and the
converge object the oracle's time for the same lattice, extrapolated from
its measured rate.
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
KERNEL_SOURCES = ("paper_1906_06327_amd/csrc/sscn_device.hpp", "paper_1906_06327_amd/csrc/sscn_lib.hip")


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
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=256)
    ap.add_argument("--precision", choices=("c128", "c64"), default="c128")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip variants and convergence")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--profile-sample", action="store_true",
                    help="run a short fixed sample for hardware-counter passes and exit: a "
                         "256 MiB device copy (counter calibration), 50 steps of the 512^2 "
                         "complex128 workload, 20 steps of the 3D complex64 workload")
    return ap.parse_args()


def profile_sample(P, torch):
    n = 256 * 1024 * 1024 // 16
    a = torch.ones(n, dtype=torch.complex128, device="cuda")
    c = torch.empty_like(a)
    for _ in range(3):
        c.copy_(a)
    torch.cuda.synchronize()
    print("profile-sample: copy 256 MiB x3 done", flush=True)
    for cfg, k in ((W.CONFIGS["c2"], 50), (W.CONFIGS["c3"], 20)):
        s = P.Solver(W.solver_params(cfg))
        s.init_state(1, W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"]), 1.0, cfg.get("d_z", 0.0))
        s.step(k)
        torch.cuda.synchronize()
        print(f"profile-sample: {cfg['nx']}x{cfg['ny']}x{cfg['nz']} {k} steps, "
              f"plan {s.solver_info()['plan']}", flush=True)
        s.close()


def timed_steps(P, torch, cfg, steps, warmup, mode=0):
    """Warm up, then time exactly `steps` steps: wall clock between two
    synchronisations, and HIP events recorded on the solver's stream (the
    current torch stream, which the solver launches on) around the same
    region.  Returns (solver, wall seconds, event milliseconds per step)."""
    s = P.Solver(W.solver_params(cfg, mode=mode), stream=torch.cuda.current_stream())
    ph = W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"])
    s.init_state(cfg.get("kind", 1), ph, cfg.get("d_xy", 1.0), cfg.get("d_z", 0.0))
    s.step(warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return s, dt, e0.elapsed_time(e1) / steps


def real_time_phase(P, torch, s, steps):
    """From the solver's current imaginary-time state, `steps` real-time
    steps (same grid and precision): wall time and the drift of the norm
    and of the full energy functional, which real time conserves up to the
    splitting error."""
    o0 = s.observables()
    s.set_mode(P.SSCN_REAL)
    s.step(64)  # the plan for real time is tuned on its first step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    o1 = s.observables()
    return {"steps": steps + 64, "ms_per_step_timed": round(dt / steps * 1e3, 6),
            "norm_drift": o1["norm"] - o0["norm"],
            "energy_full_rel_drift": (o1["energy_full"] - o0["energy_full"]) / abs(o0["energy_full"])}


def kernel_roofline(s, cfg, step_ms, nlaunch=200, traffic_key=None):
    """Average duration of the dominant kernel of a step and its algorithmic
    bandwidth.  The fused 2D plan launches one kernel per step (plus one
    final rescale per 64-step graph), so its duration is the event time of
    the timed region per step, step_ms.  The sweep plans launch several;
    each is timed over nlaunch back-to-back launches between two HIP events
    on the solver's stream (sscn_profile_kernel).  Algorithmic bytes: 2*c
    per point per axis sweep the kernel performs (one read and one write of
    the state per sweep, complex size c), i.e. 2*c*P per sweep kernel and
    2*d*c*P for the fused 2D step, which performs both sweeps of a step in
    one launch."""
    plan = s.solver_info()["plan"]
    dim = cfg["dim"]
    pts = cfg["nx"] * cfg["ny"] * (cfg["nz"] if dim == 3 else 1)
    esize = 16 if cfg.get("precision", 0) == 0 else 8
    if plan == 2:
        names = ("fused",)
        per_launch = 2 * dim * esize * pts
    else:
        names = ("x", "y", "z")[:dim]
        per_launch = 2 * esize * pts
    if plan == 2:
        ms = {"fused": step_ms}
    else:
        ms = {k: s.profile_kernel(w, nlaunch) for w, k in enumerate(names)}
    dom = max(names, key=lambda k: ms[k])
    label = "fused 2D step (H1 + x + y)" if plan == 2 else f"{dom}-sweep"
    gbs = per_launch / (ms[dom] * 1e-3) / 1e9
    kind = "fused2d" if plan == 2 else f"{dom}sweep"
    traffic = measured_traffic(traffic_key) if traffic_key and traffic_key.startswith(kind) else None
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic,
            "traffic_unit": "bytes per launch (counters)",
            "traffic_over_algorithmic": round(traffic / per_launch, 3) if traffic else None,
            "kernel": label, "plan": {1: "sweeps", 2: "fused"}.get(plan, plan),
            "x_lines_per_block": s.solver_info()["x_lines"],
            "bytes_per_launch": per_launch, "kernel_ms": {k: round(v, 6) for k, v in ms.items()},
            "timing": "events around the timed steps" if plan == 2 else "events around back-to-back launches",
            "step_ms_events": round(step_ms, 6)}


def batch_run(P, torch, steps=200):
    """The 64-instance batch: updates/s of the batched step (the plan the
    batch autotuner picks: batched sweeps or the fused step)."""
    cfgs = W.batch_instances()
    b = P.Batch(cfgs)
    for k, c in enumerate(cfgs):
        b.init_state(k, 1, W.phase_field(c["seed"], c["ny"], c["nx"]), 1.0)
    b.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pts = sum(c["nx"] * c["ny"] for c in cfgs)
    info = b.info()
    b.close()
    ups = pts * steps / dt
    return {"instances": len(cfgs), "points": pts, "updates_per_s": round(ups, 1),
            "ms_per_step": round(dt / steps * 1e3, 5),
            "plan": {1: "batched sweeps", 2: "fused"}.get(info["plan"], info["plan"]), "window": info["window"],
            "algorithmic_GBps": round(64 * ups / 1e9, 1), "frac_of_8TBps": round(64 * ups / 8e12, 4)}


def converge_run(P, torch, cfg, precision, max_steps=3000000):
    """Imaginary time from Eq. (fun) to |mu_n - mu_{n-1}| < 1e-8 at two
    consecutive checks 0.1 time units apart with the vortex count unchanged
    (sscn_converge; complex64 bulk switches to complex128 at its plateau)."""
    s = P.Solver(W.solver_params(cfg, precision=precision))
    ph = W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"])
    chk = max(1, int(round(0.1 / cfg["dt"])))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.init_state(1, ph, 1.0)
    steps, ok = s.converge(max_steps, check_every=chk, tol=1e-8, switch_tol=3e-7)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ob = s.observables()
    out = {"precision": "c128" if precision == 0 else "c64 bulk -> c128", "steps": steps,
           "converged": ok, "wall_s": round(wall, 3), "mu": ob["mu"], "energy": ob["energy"],
           "vortices": s.vortex_count(), "fp32_steps": s.switch_step if precision == 1 else 0}
    s.close()
    return out


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


def cpu_baseline(cfg, seconds):
    """The FP64 oracle as it stands on the host cores, on a bounded sample
    (consecutive steps of the same workload from the same initial state),
    and the same on one thread."""
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rate, steps, dt = oracle_rate(cfg, seconds)
    out = {"value": round(rate, 1), "unit": "updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{steps} consecutive imaginary-time steps of the 512x512 complex128 "
                     f"workload ({dt:.1f} s), OpenMP over lines with {threads} threads"}
    if _omp_threads(1):
        r1, s1, d1 = oracle_rate(cfg, seconds / 2, chunk=5)
        _omp_threads(threads)
        out["single_thread"] = {"value": round(r1, 1), "unit": "updates/s", "cores": 1,
                                "sample": f"{s1} consecutive steps of the same workload ({d1:.1f} s)"}
    return out


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """GB/s of a plain device-to-device copy (read + write counted), timed
    with HIP events: the achievable HBM bandwidth the kernels are also
    compared with."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus > 1 or world > 1:
        print(f"bench.py measures one GPU only: this solver has no multi-GPU path "
              f"(asked for --gpus {a.gpus}, WORLD_SIZE {world}).", flush=True)
        sys.exit(2)
    import torch
    import paper_1906_06327_amd as P
    P.lib()
    cfg = dict(W.CONFIGS["c2"], precision=0 if a.precision == "c128" else 1)
    torch.cuda.set_device(0)
    if a.profile_sample:
        profile_sample(P, torch)
        return

    s, dt, step_ms = timed_steps(P, torch, cfg, a.steps, a.warmup)
    pts = cfg["nx"] * cfg["ny"]
    value = pts * a.steps / dt
    roof = kernel_roofline(s, cfg, step_ms, traffic_key=f"fused2d_512_{a.precision}")
    rt_phase = None if a.no_extras else real_time_phase(P, torch, s, 10000)
    s.close()
    copy_gbs = copy_bandwidth(torch)
    roof["copy_GBps"] = round(copy_gbs, 1)
    roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)

    out = {
        "metric": "grid-point updates/s per SSCN step (% HBM roofline) + time-to-converged lattice",
        "value": round(value, 1), "unit": "updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(dt / a.steps * 1e3, 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if a.precision == "c128" else "f32",
        "data": "synthetic (one-vortex random-phase initial state, seed 13)",
        "config": {"workload": "2D rotating GP, 512x512 on [-12.8,12.8)^2, gamma=1, nu=1.05, "
                               "g=1000, Omega=0.9, dt=5e-4, imaginary time, renormalised each step",
                   "grid": [cfg["nx"], cfg["ny"]], "precision": a.precision,
                   "parallelism": "single GPU"},
        "roofline": roof,
    }
    if not a.no_extras:
        variants = {}
        c64 = dict(W.CONFIGS["c2"], precision=1)
        s, dt, sm = timed_steps(P, torch, c64, 5000, 256)
        variants["c2_complex64"] = {"updates_per_s": round(pts * 5000 / dt, 1),
                                    "ms_per_step": round(dt / 5000 * 1e3, 6),
                                    "roofline": kernel_roofline(s, c64, sm)}
        s.close()
        s, dt, _ = timed_steps(P, torch, W.CONFIGS["c2"], 5000, 256, mode=1)
        variants["c2_real_time_complex128"] = {"updates_per_s": round(pts * 5000 / dt, 1),
                                               "ms_per_step": round(dt / 5000 * 1e3, 6)}
        s.close()
        c3 = W.CONFIGS["c3"]
        s, dt, sm = timed_steps(P, torch, c3, 1000, 64)
        p3 = c3["nx"] * c3["ny"] * c3["nz"]
        variants["c3_3d_complex64"] = {"updates_per_s": round(p3 * 1000 / dt, 1),
                                       "ms_per_step": round(dt / 1000 * 1e3, 6),
                                       "roofline": kernel_roofline(s, c3, sm, 100,
                                                                   traffic_key="xsweep_3d_256x256x64_c64")}
        variants["c3_3d_complex64"]["then_real_time"] = real_time_phase(P, torch, s, 1000)
        s.close()
        variants["c2_then_real_time"] = rt_phase
        variants["c4_batch_64_instances_complex128"] = batch_run(P, torch)
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
            rate, steps, dt = oracle_rate(c1, 3.0)
            conv["c128"]["oracle_extrapolated_s"] = round(conv["c128"]["steps"] * c1["nx"] * c1["ny"] / rate, 1)
            conv["c128"]["oracle_sample"] = f"{steps} oracle steps in {dt:.1f} s on the host cores"
        out["converge"] = conv
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(W.CONFIGS["c2"], a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
