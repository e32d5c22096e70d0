"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Both sides start from the same seeded inputs (workloads module) and are
compared element by element.  Tolerances: relative L2 error of the state
<= 1e-10 for complex128 sweeps and <= 1e-5 for complex64 sweeps with FP64
reductions; observables to the same relative bounds.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5


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


def both(P, cfg):
    """(GPU solver, oracle params) for one parameter dict."""
    sp = W.solver_params(cfg)
    return P.Solver(sp), O.make_params(**sp)


def check_obs(go, oo, tol):
    errs = {}
    for k in ("norm", "mu", "energy", "mu_full", "energy_full", "mu_4th", "energy_4th", "rms_x", "rms_y",
              "rms_r"):
        errs[k] = abs(go[k] - oo[k]) / max(1.0, abs(oo[k]))
        assert errs[k] <= tol, (k, go[k], oo[k])
    print("[gpu-parity] observable errors vs oracle: " +
          ", ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)


def announce(msg):
    print(f"[gpu-parity] {msg}", flush=True)


# --------------------------------------------------------------------------

def test_init_state_matches_oracle(P):
    for cfg in (W.CONFIGS["c1"], dict(W.CONFIGS["c3"], nx=48, ny=40, nz=20, precision=0)):
        announce(f"init dim={cfg['dim']}")
        s, op = both(P, cfg)
        ph = W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"])
        dz = cfg.get("d_z", 0.0)
        s.init_state(1, ph, cfg["d_xy"], dz)
        ref = O.init_state(op, 1, ph, cfg["d_xy"], dz if dz > 0 else None)
        assert rel(s.get_state(), ref) <= 1e-14
        s.init_state(0, None, 1.3, dz)
        ref = O.init_state(op, 0, None, 1.3, dz if dz > 0 else None)
        assert rel(s.get_state(), ref) <= 1e-14
        s.close()


def test_seeded_init_state_matches_oracle(P):
    """The device's counter-based random phase gives the oracle's numbers bit
    for bit (integer hashing), and the seeded initial state of Eq. (fun)
    matches the oracle's from those numbers, in 2D and 3D."""
    announce("seeded phase field")
    got = P.phase_field_seed(13, 37, 53).cpu().numpy()
    assert np.array_equal(got, O.splitmix_phase(13, 37, 53))
    big = P.phase_field_seed(2**63 + 5, 200, 256).cpu().numpy()
    assert np.array_equal(big[::17, ::13], O.splitmix_phase(2**63 + 5, 200, 256)[::17, ::13])
    for cfg in (dict(W.CONFIGS["c1"], nx=96, ny=80), dict(W.CONFIGS["c3"], nx=48, ny=40, nz=20, precision=0)):
        announce(f"seeded init dim={cfg['dim']}")
        s, op = both(P, cfg)
        dz = cfg.get("d_z", 0.0)
        for seed in (13, 7):
            s.init_state_seed(1, seed, cfg["d_xy"], dz)
            ref = O.init_state(op, 1, O.splitmix_phase(seed, cfg["ny"], cfg["nx"]), cfg["d_xy"],
                               dz if dz > 0 else None)
            assert rel(s.get_state(), ref) <= 1e-14
        s.init_state_seed(0, 13, 1.3, dz, random_phase=False)
        ref = O.init_state(op, 0, None, 1.3, dz if dz > 0 else None)
        assert rel(s.get_state(), ref) <= 1e-14
        s.close()


def test_config1_full_run_matches_oracle(P):
    """128^2, g = 100, Omega = 0.6, dt = 1e-3, 1000 imaginary-time steps."""
    cfg = W.CONFIGS["c1"]
    announce("c1 1000 steps")
    s, op = both(P, cfg)
    ph = W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"])
    s.init_state(1, ph, 1.0)
    ref = O.init_state(op, 1, ph, 1.0)
    assert s.solver_info()["window"][0] > 0  # windowed kernels, not the fallback
    s.step(cfg["steps"])
    ref = O.step(op, ref, cfg["steps"])
    got = s.get_state()
    assert rel(got, ref) <= TOL64
    check_obs(s.observables(), O.observables(op, ref), TOL64)
    assert s.vortex_count() == O.vortex_count(op, ref)
    s.close()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("shape", [(100, 77), (64, 64), (130, 9), (5, 200)])
def test_ragged_2d(P, mode, shape):
    nx, ny = shape
    announce(f"ragged 2d {shape} mode={mode}")
    cfg = dict(dim=2, nx=nx, ny=ny, nz=1, hx=0.11, hy=0.09, hz=0.1, gamma=1.0, nu=1.1,
               lam=1.0, g=60.0, omega=0.55, dt=2e-3, mode=mode, precision=0)
    s, op = both(P, cfg)
    psi0 = W.random_field(11, (ny, nx)) / np.sqrt(0.11 * 0.09)
    s.set_state(psi0)
    s.step(150)
    ref = O.step(op, psi0, 150)
    assert rel(s.get_state(), ref) <= TOL64
    s.close()


@pytest.mark.parametrize("mode", [0, 1])
def test_ragged_3d(P, mode):
    announce(f"ragged 3d mode={mode}")
    cfg = dict(dim=3, nx=37, ny=30, nz=21, hx=0.2, hy=0.22, hz=0.15, gamma=1.0, nu=1.05,
               lam=2.0, g=40.0, omega=0.4, dt=2e-3, mode=mode, precision=0)
    s, op = both(P, cfg)
    psi0 = W.random_field(12, (21, 30, 37)) / np.sqrt(0.2 * 0.22 * 0.15)
    s.set_state(psi0)
    s.step(70)
    ref = O.step(op, psi0, 70)
    assert rel(s.get_state(), ref) <= TOL64
    s.close()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("mode", [0, 1])
def test_complex64_bulk(P, dim, mode):
    announce(f"c64 dim={dim} mode={mode}")
    if dim == 2:
        cfg = dict(dim=2, nx=96, ny=90, nz=1, hx=0.1, hy=0.1, hz=0.1, gamma=1.0, nu=1.05,
                   lam=1.0, g=100.0, omega=0.6, dt=1e-3, mode=mode, precision=1)
        shp = (90, 96)
    else:
        cfg = dict(dim=3, nx=40, ny=44, nz=24, hx=0.2, hy=0.2, hz=0.2, gamma=1.0, nu=1.0,
                   lam=4.0, g=200.0, omega=0.5, dt=5e-4, mode=mode, precision=1)
        shp = (24, 44, 40)
    s, op = both(P, cfg)
    ph = W.phase_field(5, cfg["ny"], cfg["nx"])
    s.init_state(1, ph, 1.0, 0.5)
    ref = O.init_state(op, 1, ph, 1.0, 0.5)
    s.step(300)
    ref = O.step(op, ref, 300)
    got = s.get_state()
    assert got.shape == shp
    assert rel(got.astype(np.complex128), ref) <= TOL32
    check_obs(s.observables(), O.observables(op, ref), TOL32)
    s.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_exact_whole_line_path(P, dim):
    """Parameters whose decay bound needs a window beyond 32 rows run the
    exact whole-line kernels."""
    announce(f"exact path dim={dim}")
    if dim == 2:
        cfg = dict(dim=2, nx=50, ny=45, nz=1, hx=0.1, hy=0.1, hz=0.1, gamma=1.0, nu=1.0,
                   lam=1.0, g=20.0, omega=0.3, dt=0.2, mode=0, precision=0)
        shp = (45, 50)
    else:
        cfg = dict(dim=3, nx=20, ny=22, nz=18, hx=0.3, hy=0.3, hz=0.1, gamma=1.0, nu=1.0,
                   lam=3.0, g=20.0, omega=0.3, dt=0.1, mode=0, precision=0)
        shp = (18, 22, 20)
    s, op = both(P, cfg)
    assert s.solver_info()["window"] == [0, 0, 0]
    psi0 = W.random_field(13, shp)
    s.set_state(psi0)
    s.step(20)
    ref = O.step(op, psi0, 20)
    assert rel(s.get_state(), ref) <= TOL64
    s.close()


def test_config2_full_size(P):
    """512^2 on [-12.8, 12.8)^2, g = 1000, Omega = 0.9, dt = 5e-4: a stretch
    of the imaginary-time phase and of the real-time phase at full size."""
    cfg = W.CONFIGS["c2"]
    announce("c2 512^2 imag 80 + real 40 (c128)")
    s, op = both(P, cfg)
    ph = W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"])
    s.init_state(1, ph, 1.0)
    ref = O.init_state(op, 1, ph, 1.0)
    s.step(80)
    ref = O.step(op, ref, 80)
    assert rel(s.get_state(), ref) <= TOL64
    s.set_mode(1)
    opr = O.make_params(**W.solver_params(cfg, mode=1))
    s.step(40)
    ref = O.step(opr, ref, 40)
    assert rel(s.get_state(), ref) <= TOL64
    check_obs(s.observables(), O.observables(opr, ref), TOL64)
    s.close()


def test_config2_complex64_variant(P):
    cfg = dict(W.CONFIGS["c2"], precision=1)
    announce("c2 512^2 imag 80 (c64)")
    s, op = both(P, cfg)
    ph = W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"])
    s.init_state(1, ph, 1.0)
    ref = O.init_state(op, 1, ph, 1.0)
    s.step(80)
    ref = O.step(op, ref, 80)
    assert rel(s.get_state().astype(np.complex128), ref) <= TOL32
    check_obs(s.observables(), O.observables(op, ref), TOL32)
    s.close()


def test_config3_full_size_complex64(P):
    """256 x 256 x 64, complex64 sweeps with FP64 norm: a few steps at full
    size against the FP64 oracle."""
    cfg = W.CONFIGS["c3"]
    announce("c3 256x256x64 c64, 6 steps")
    s, op = both(P, cfg)
    ph = W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"])
    s.init_state(1, ph, 1.0, cfg["d_z"])
    ref = O.init_state(op, 1, ph, 1.0, cfg["d_z"])
    s.step(6)
    ref = O.step(op, ref, 6)
    assert rel(s.get_state().astype(np.complex128), ref) <= TOL32
    check_obs(s.observables(), O.observables(op, ref), TOL32)
    s.close()


def test_real_time_norm_conserved(P):
    announce("real-time unitarity")
    cfg = dict(dim=2, nx=128, ny=128, nz=1, hx=0.1, hy=0.1, hz=0.1, gamma=1.0, nu=1.0,
               lam=1.0, g=100.0, omega=0.6, dt=1e-3, mode=1, precision=0)
    s = P.Solver(W.solver_params(cfg))
    s.init_state(1, W.phase_field(3, 128, 128), 1.0)
    n0 = s.observables()["norm"]
    s.step(3000)
    assert abs(s.observables()["norm"] - n0) <= 1e-12
    s.close()


def test_real_time_energy_excursion_is_first_order_in_dt(P):
    """Real time on the full 512^2 workload from a partly relaxed state: the
    norm stays at 1 to rounding and the largest excursion of the
    full-functional energy over 2 time units halves with dt (the splitting
    is first order; the continuum dynamics conserve E)."""
    announce("real-time energy excursion, 512^2")
    cfg = W.CONFIGS["c2"]
    s = P.Solver(W.solver_params(cfg))
    s.init_state(1, W.phase_field(13, cfg["ny"], cfg["nx"]), 1.0)
    s.step(4000)
    psi0 = s.get_state()
    s.close()
    dev = []
    for dt in (cfg["dt"], cfg["dt"] / 2):
        r = P.Solver(W.solver_params(cfg, mode=1, dt=dt))
        r.set_state(psi0)
        o0 = r.observables()
        mx, k = 0.0, int(round(0.05 / dt))
        for _ in range(40):
            r.step(k)
            o = r.observables()
            mx = max(mx, abs(o["energy_full"] - o0["energy_full"]))
            assert abs(o["norm"] - o0["norm"]) <= 1e-12
        dev.append(mx)
        r.close()
    assert dev[0] < 1e-3 * abs(o0["energy_full"])
    assert 1.8 <= dev[0] / dev[1] <= 2.4, dev


def test_observables_and_vortex_count_match_oracle(P):
    announce("observables / vortex count")
    cfg = dict(dim=2, nx=128, ny=128, nz=1, hx=0.1, hy=0.1, hz=0.1, gamma=1.0, nu=1.2,
               lam=1.0, g=80.0, omega=0.45, dt=1e-3, mode=0, precision=0)
    s, op = both(P, cfg)
    x = -6.4 + 0.1 * np.arange(128)
    Y, X = np.meshgrid(x, x, indexing="ij")
    Z = X + 1j * Y
    psi = np.exp(-(X ** 2 + Y ** 2) / 8).astype(complex)
    for z0 in [0.03 + 0.02j] + [1.5 * np.exp(1j * (np.pi / 3 * k + 0.1)) for k in range(6)]:
        psi = psi * (Z - z0) / np.sqrt(np.abs(Z - z0) ** 2 + 0.04)
    psi = psi * np.exp(0.3j * X)
    psi[0, :] = 0
    psi[:, 0] = 0
    s.set_state(psi)
    check_obs(s.observables(), O.observables(op, psi), 1e-12)
    assert s.vortex_count() == O.vortex_count(op, psi) == 7
    s.close()


def test_deterministic_and_restartable(P):
    announce("determinism / restart")
    cfg = dict(W.CONFIGS["c1"])
    sp = W.solver_params(cfg)
    ph = W.phase_field(7, 128, 128)
    a = P.Solver(sp)
    a.init_state(1, ph, 1.0)
    a.step(300)
    ra = a.get_state()
    b = P.Solver(sp)
    b.init_state(1, ph, 1.0)
    b.step(100)
    mid = b.get_state()
    b.close()
    c = P.Solver(sp)
    c.set_state(mid)
    c.step(200)
    rc = c.get_state()
    a2 = P.Solver(sp)
    a2.init_state(1, ph, 1.0)
    a2.step(300)
    assert np.array_equal(a2.get_state(), ra)       # run-to-run bitwise
    # restart bitwise: the rescale that ends a call (k_rescale) and the one
    # folded into the next step sum the norm partials in the same order, so
    # a run restarted from a saved state repeats the uninterrupted run
    assert np.array_equal(rc, ra)
    for s in (a, a2, c):
        s.close()


def test_precision_upcast(P):
    """complex64 bulk, then upcast to complex128 and continue (FP64
    refinement); the continuation matches the oracle run from the upcast
    state."""
    announce("c64 -> c128 upcast")
    cfg = dict(dim=2, nx=96, ny=96, nz=1, hx=0.1, hy=0.1, hz=0.1, gamma=1.0, nu=1.0,
               lam=1.0, g=100.0, omega=0.6, dt=1e-3, mode=0, precision=1)
    s = P.Solver(W.solver_params(cfg))
    s.init_state(1, W.phase_field(9, 96, 96), 1.0)
    s.step(200)
    mid = s.get_state().astype(np.complex128)
    s.set_mode(0, 0)
    assert s.psi.dtype.itemsize == 16
    assert np.array_equal(s.get_state(), mid)
    s.step(200)
    op = O.make_params(**W.solver_params(cfg, precision=0))
    assert rel(s.get_state(), O.step(op, mid, 200)) <= TOL64
    s.close()


# --------------------------------------------------------------------------
# Both step plans (separate sweeps; fused 2D tiles) against the oracle.

@pytest.mark.parametrize("plan", [1, 2])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("prec,shape", [(0, (100, 77)), (0, (130, 47)), (1, (96, 70)), (0, (33, 200)),
                                        (0, (129, 40)), (1, (129, 52))])
def test_plans_2d(P, plan, mode, prec, shape):
    """nx = 129 gives 16 lines per x-sweep block, nx * L > 2048, so the
    x-sweep stages 16 points per thread (the others 8)."""
    nx, ny = shape
    announce(f"plan={plan} mode={mode} prec={prec} shape={shape}")
    cfg = dict(dim=2, nx=nx, ny=ny, nz=1, hx=0.11, hy=0.09, hz=0.1, gamma=1.0, nu=1.1,
               lam=1.0, g=60.0, omega=0.55, dt=2e-3, mode=mode, precision=prec)
    s, op = both(P, cfg)
    s.set_plan(plan)
    psi0 = W.random_field(21, (ny, nx)) / np.sqrt(0.11 * 0.09)
    s.set_state(psi0)
    s.step(131)  # odd: exercises the buffer hand-back
    assert s.solver_info()["plan"] == plan
    ref = O.step(op, psi0, 131)
    got = s.get_state().astype(np.complex128)
    assert rel(got, ref) <= (TOL64 if prec == 0 else TOL32)
    s.close()


@pytest.mark.parametrize("tile", [0, 1, 2])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("prec,shape", [(0, (100, 77)), (1, (96, 70)), (0, (33, 200)), (0, (129, 40))])
def test_fused_tile_shapes(P, tile, mode, prec, shape, monkeypatch):
    """The fused step's tile shapes (32 x 32, 32 x 16 and 16 x 16, fixed
    through SSCN_FUSED_TILE) against the oracle on ragged grids, over
    graph-replayed steps (an odd count: the buffer hand-back) and, bit for
    bit, the same steps launched one at a time."""
    nx, ny = shape
    announce(f"fused tile={tile} mode={mode} prec={prec} shape={shape}")
    monkeypatch.setenv("SSCN_FUSED_TILE", str(tile))
    cfg = dict(dim=2, nx=nx, ny=ny, nz=1, hx=0.11, hy=0.09, hz=0.1, gamma=1.0, nu=1.1,
               lam=1.0, g=60.0, omega=0.55, dt=2e-3, mode=mode, precision=prec)
    psi0 = W.random_field(22, (ny, nx)) / np.sqrt(0.11 * 0.09)
    s, op = both(P, cfg)
    s.set_plan(2)
    s.set_state(psi0)
    s.step(131)
    info = s.solver_info()
    assert info["plan"] == 2 and info["fused_tile"] == [[32, 32], [32, 16], [16, 16]][tile], info
    ref = O.step(op, psi0, 131)
    got = s.get_state()
    assert rel(got.astype(np.complex128), ref) <= (TOL64 if prec == 0 else TOL32)
    s.close()
    d = P.Solver(W.solver_params(cfg))
    d.set_plan(2)
    d.set_state(psi0)
    for _ in range(131):
        d.step(1)
    assert np.array_equal(d.get_state(), got)
    d.close()


@pytest.mark.parametrize("plan", [1, 2])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("prec", [0, 1])
def test_large_h1_arguments(P, plan, mode, prec):
    """dt times the potential reaches 0.86 at the box edge, so the threads
    holding edge points take the library branch of the H1 factor (|dt w| >
    1/4) while the others use its series; both must match the oracle."""
    nx, ny = 100, 77
    announce(f"large H1 arguments plan={plan} mode={mode} prec={prec}")
    cfg = dict(dim=2, nx=nx, ny=ny, nz=1, hx=0.2, hy=0.2, hz=0.1, gamma=1.0, nu=1.1,
               lam=1.0, g=60.0, omega=0.55, dt=1e-2, mode=mode, precision=prec)
    s, op = both(P, cfg)
    s.set_plan(plan)
    x = -nx * 0.1 + 0.2 * np.arange(nx)
    assert 1e-2 * 0.5 * x.max() ** 2 > 0.25  # the library branch is exercised
    psi0 = W.random_field(23, (ny, nx)) / np.sqrt(0.2 * 0.2)
    s.set_state(psi0)
    s.step(60)
    assert s.solver_info()["plan"] == plan
    ref = O.step(op, psi0, 60)
    got = s.get_state().astype(np.complex128)
    assert rel(got, ref) <= (TOL64 if prec == 0 else TOL32)
    s.close()


@pytest.mark.parametrize("plan", [1, 2])
def test_plans_config2_full_size(P, plan):
    cfg = W.CONFIGS["c2"]
    announce(f"c2 full size plan={plan}")
    s, op = both(P, cfg)
    s.set_plan(plan)
    ph = W.phase_field(cfg["seed"], cfg["ny"], cfg["nx"])
    s.init_state(1, ph, 1.0)
    s.step(70)
    ref = O.step(op, O.init_state(op, 1, ph, 1.0), 70)
    assert rel(s.get_state(), ref) <= TOL64
    s.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_autotuner_cache_file_and_x_lines(P, dim, tmp_path, monkeypatch):
    """A choice read from the SSCN_TUNE_CACHE file is applied (plan and
    x-sweep lines per block), every admissible lines-per-block value gives
    the oracle's result, and a tuned choice is written back to the file."""
    if dim == 2:
        cfg = dict(dim=2, nx=70, ny=58, nz=1, hx=0.15, hy=0.17, hz=0.1, gamma=1.0, nu=1.1, lam=1.0,
                   g=40.0, omega=0.5, dt=2e-3, mode=0, precision=0)
    else:
        cfg = dict(dim=3, nx=46, ny=38, nz=22, hx=0.3, hy=0.3, hz=0.35, gamma=1.0, nu=1.1, lam=2.0,
                   g=30.0, omega=0.4, dt=2e-3, mode=0, precision=0)
    path = tmp_path / "tune.json"
    monkeypatch.setenv("SSCN_TUNE_CACHE", str(path))
    ph = W.phase_field(5, cfg["ny"], cfg["nx"])
    op = O.make_params(**cfg)
    ref = O.step(op, O.init_state(op, 1, ph, 1.0), 9)
    probe = P.Solver(cfg)
    win, lmax = probe.solver_info()["window"][0], probe.solver_info()["x_lines"]
    probe.close()
    key = "gfx950|%dd|%dx%dx%d|c128|imag|W%d" % (dim, cfg["nx"], cfg["ny"], cfg["nz"] if dim == 3 else 1, win)
    for xl in sorted({1, max(1, lmax // 2), lmax}):
        announce(f"tune cache dim={dim} x_lines={xl}")
        path.write_text('{\n  "%s": {"plan": 1, "x_lines": %d, "ms_per_step": 0.0}\n}\n' % (key, xl))
        monkeypatch.setenv("SSCN_TUNE_CACHE", str(path) + ".%d" % xl)  # a new name forces a re-read
        path.rename(str(path) + ".%d" % xl)
        s = P.Solver(cfg)
        s.init_state(1, ph, 1.0)
        s.step(9)
        info = s.solver_info()
        assert info["plan"] == 1 and info["x_lines"] == xl, info
        assert rel(s.get_state(), ref) <= TOL64
        s.close()
    # an untuned shape is timed and written to the file
    other = dict(cfg, nx=cfg["nx"] + 6)
    out = tmp_path / "fresh.json"
    monkeypatch.setenv("SSCN_TUNE_CACHE", str(out))
    s = P.Solver(other)
    s.init_state(1, W.phase_field(5, other["ny"], other["nx"]), 1.0)
    s.step(3)
    info = s.solver_info()
    s.close()
    text = out.read_text()
    assert "%dx%d" % (other["nx"], other["ny"]) in text and '"x_lines": %d' % info["x_lines"] in text, text


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("nx", [128, 129])
def test_x_sweep_staging_depths(P, nx, prec, tmp_path, monkeypatch):
    """With the largest lines-per-block value (forced through the tune
    cache) nx = 128 stages 8 points per x-sweep thread (nx * L = 2048) and
    nx = 129 stages 16 (nx * L = 2064); both match the oracle."""
    cfg = dict(dim=2, nx=nx, ny=41, nz=1, hx=0.12, hy=0.15, hz=0.1, gamma=1.0, nu=1.1, lam=1.0,
               g=40.0, omega=0.5, dt=2e-3, mode=0, precision=prec)
    monkeypatch.setenv("SSCN_TUNE_CACHE", str(tmp_path / "none.json"))
    probe = P.Solver(cfg)
    win, lmax = probe.solver_info()["window"][0], probe.solver_info()["x_lines"]
    probe.close()
    assert lmax == 16, lmax
    key = "gfx950|2d|%dx%dx1|%s|imag|W%d" % (nx, cfg["ny"], "c128" if prec == 0 else "c64", win)
    path = tmp_path / "tune.json"
    path.write_text('{\n  "%s": {"plan": 1, "x_lines": %d, "ms_per_step": 0.0}\n}\n' % (key, lmax))
    monkeypatch.setenv("SSCN_TUNE_CACHE", str(path))
    announce(f"x-sweep staging nx={nx} prec={prec} x_lines={lmax}")
    ph = W.phase_field(6, cfg["ny"], nx)
    op = O.make_params(**cfg)
    ref = O.step(op, O.init_state(op, 1, ph, 1.0), 25)
    s = P.Solver(cfg)
    s.init_state(1, ph, 1.0)
    s.step(25)
    info = s.solver_info()
    assert info["plan"] == 1 and info["x_lines"] == lmax, info
    assert rel(s.get_state().astype(np.complex128), ref) <= (TOL64 if prec == 0 else TOL32)
    s.close()


@pytest.mark.parametrize("dim,plan,mode", [(2, 2, 0), (2, 1, 0), (2, 1, 1), (3, 1, 0)])
def test_profile_kernel_leaves_state_alone(P, dim, plan, mode):
    """Per-kernel timing runs the step's kernels into scratch: positive
    durations for the kernels the plan has, an error for the others, and the
    state and the next steps unchanged (still equal to the oracle's)."""
    if dim == 2:
        cfg = dict(dim=2, nx=100, ny=90, nz=1, hx=0.12, hy=0.13, hz=0.1, gamma=1.0, nu=1.1, lam=1.0,
                   g=50.0, omega=0.5, dt=2e-3, mode=mode, precision=0)
    else:
        cfg = dict(dim=3, nx=40, ny=36, nz=30, hx=0.3, hy=0.3, hz=0.3, gamma=1.0, nu=1.1, lam=2.0,
                   g=30.0, omega=0.4, dt=2e-3, mode=mode, precision=0)
    announce(f"profile_kernel dim={dim} plan={plan} mode={mode}")
    s, op = both(P, cfg)
    s.set_plan(plan)
    ph = W.phase_field(6, cfg["ny"], cfg["nx"])
    s.init_state(1, ph, 1.0)
    s.step(5)
    kernels = [0] if plan == 2 else ([0, 1] if dim == 2 else [0, 1, 2])
    for which in kernels:
        assert s.profile_kernel(which, 20) > 0
    for which in set(range(3)) - set(kernels):
        with pytest.raises(P.SSCNError):
            s.profile_kernel(which, 5)
    s.step(5)
    ref = O.step(op, O.init_state(op, 1, ph, 1.0), 10)
    assert rel(s.get_state(), ref) <= TOL64
    s.close()


def test_fused_plan_rejected_in_3d(P):
    cfg = dict(dim=3, nx=20, ny=20, nz=20, hx=0.2, hy=0.2, hz=0.2, gamma=1.0, nu=1.0, lam=2.0,
               g=10.0, omega=0.3, dt=1e-3, mode=0, precision=0)
    s = P.Solver(cfg)
    with pytest.raises(P.SSCNError):
        s.set_plan(2)
    s.close()


def test_converge_fp64_and_mixed_precision(P):
    """sscn_converge: the FP64 run stops at the criterion and its state is the
    oracle's after the same number of steps; the complex64 run switches to
    complex128 at its plateau and reaches the same converged mu."""
    announce("converge fp64 / c64->c128")
    cfg = dict(dim=2, nx=56, ny=52, nz=1, hx=0.25, hy=0.25, hz=0.1, gamma=1.0, nu=1.1,
               lam=1.0, g=25.0, omega=0.35, dt=0.01, mode=0, precision=0)
    ph = W.phase_field(61, 52, 56)
    s, op = both(P, cfg)
    s.init_state(1, ph, 1.0)
    steps, ok = s.converge(200000, check_every=20, tol=1e-9)
    assert ok and steps < 200000
    ref = O.step(op, O.init_state(op, 1, ph, 1.0), steps)
    assert rel(s.get_state(), ref) <= TOL64
    mu64 = s.observables()["mu"]
    s.close()
    s32 = P.Solver(W.solver_params(cfg, precision=1))
    s32.init_state(1, ph, 1.0)
    steps32, ok32 = s32.converge(200000, check_every=20, tol=1e-9, switch_tol=1e-6)
    assert ok32 and s32.params.precision == 0 and s32.psi.dtype.itemsize == 16
    assert 0 < s32.switch_step < steps32 and s.switch_step == -1
    assert abs(s32.observables()["mu"] - mu64) < 1e-7
    s32.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("src_shape,dst_shape", [((30, 40), (50, 64)), ((50, 64), (30, 40)),
                                                 ((30, 64), (50, 40)), ((10, 16, 20), (14, 20, 28)),
                                                 ((14, 20, 28), (10, 16, 20))])
def test_embed_state_matches_oracle(P, prec, src_shape, dst_shape):
    """Centred embedding (continuation start) against the oracle: pure data
    movement, so bit-exact; an odd size difference is rejected."""
    import torch
    announce(f"embed {src_shape} -> {dst_shape} prec={prec}")
    rng = np.random.default_rng(len(src_shape) * 100 + src_shape[-1])
    a = rng.standard_normal(src_shape) + 1j * rng.standard_normal(src_shape)
    dt = torch.complex128 if prec == 0 else torch.complex64
    src = torch.tensor(a).to(dt).cuda()
    dst = torch.full(dst_shape, 7.0 + 7.0j, dtype=dt, device="cuda")
    P.embed_state(src, dst)
    ref = O.embed(src.cpu().numpy().astype(np.complex128), dst_shape)
    assert np.array_equal(dst.cpu().numpy().astype(np.complex128), ref)
    bad = torch.zeros(tuple(n + (1 if k == 0 else 0) for k, n in enumerate(dst_shape)), dtype=dt, device="cuda")
    with pytest.raises(P.SSCNError):
        P.embed_state(src, bad)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", [(37, 29, 11), (64, 64, 32)])
def test_extend_z_matches_oracle(P, prec, shape):
    """The 3D product start (a 2D field times the normalised z Gaussian of
    Eq. (fun)) against the oracle; the extended oracle initial state, walls
    zeroed by the handle, steps like the handle's own 3D initial state."""
    import torch
    nx, ny, nz = shape
    announce(f"extend_z {shape} prec={prec}")
    rng = np.random.default_rng(nx + ny + nz)
    a = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    dt = torch.complex128 if prec == 0 else torch.complex64
    xy = torch.tensor(a).to(dt).cuda()
    dst = torch.full((nz, ny, nx), 7.0 + 7.0j, dtype=dt, device="cuda")
    hz, d_z = 0.17, 0.6
    P.extend_z(xy, dst, hz, d_z)
    ref = O.extend_z(xy.cpu().numpy(), nz, hz, d_z)
    assert rel(dst.cpu().numpy(), ref) <= (1e-15 if prec == 0 else 1e-7)
    with pytest.raises(P.SSCNError):
        P.extend_z(xy, dst, 0.0, d_z)
    # through a handle: the extended 2D Eq. (fun) state equals the 3D one
    cfg = dict(dim=3, nx=nx, ny=ny, nz=nz, hx=0.3, hy=0.3, hz=hz, gamma=1.0, nu=1.0, lam=1.0 / d_z ** 2, g=20.0,
               omega=0.4, dt=2e-3, mode=0, precision=prec)
    s = P.Solver(cfg)
    s2 = P.Solver(dict(cfg, dim=2, nz=1))
    ph = W.phase_field(3, ny, nx)
    s2.init_state(1, ph, 1.0)
    P.extend_z(s2.psi, s.psi, hz, d_z)
    s.set_state_device()
    s.step(5)
    s3 = P.Solver(cfg)
    s3.init_state(1, ph, 1.0, d_z)
    s3.step(5)
    assert rel(s.get_state(), s3.get_state()) <= (1e-13 if prec == 0 else 2e-6)
    for x in (s, s2, s3):
        x.close()


@pytest.mark.parametrize("dim,prec", [(2, 0), (2, 1), (3, 0), (3, 1)])
def test_density_profiles_match_oracle(P, dim, prec):
    """Every density output of sscn_density against the oracle's definition
    on the same (stepped, ragged) state; 2D handles reject the z profiles."""
    announce(f"density profiles dim={dim} prec={prec}")
    if dim == 2:
        cfg = dict(dim=2, nx=70, ny=53, nz=1, hx=0.15, hy=0.17, hz=0.1, gamma=1.0, nu=1.1, lam=1.0, g=30.0,
                   omega=0.4, dt=2e-3, mode=0, precision=prec)
    else:
        cfg = dict(dim=3, nx=34, ny=27, nz=19, hx=0.3, hy=0.3, hz=0.35, gamma=1.0, nu=1.1, lam=2.0, g=20.0,
                   omega=0.4, dt=2e-3, mode=0, precision=prec)
    s, op = both(P, cfg)
    s.init_state(1, W.phase_field(4, cfg["ny"], cfg["nx"]), 1.0)
    s.step(7)
    psi = s.get_state().astype(np.complex128)
    tol = 1e-13 if prec == 0 else 1e-6
    for kind in O.DENSITY_KINDS:
        if dim == 2 and kind in ("z", "cut_z"):
            with pytest.raises(P.SSCNError):
                s.density(kind)
            continue
        got = s.density(kind).cpu().numpy()
        ref = O.density(op, psi, kind)
        assert got.shape == ref.shape, kind
        assert np.max(np.abs(got - ref)) <= tol * max(1.0, np.max(np.abs(ref))), kind
    s.close()
