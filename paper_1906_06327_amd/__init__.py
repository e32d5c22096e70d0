"""Python binding of the MI355X SSCN library (libsscn.so, C ABI in include/sscn.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  PyTorch supplies the device memory (the state tensor) and the
stream.  The binding refuses to run when the compiled library is missing; it
has no fallback of any kind.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsscn.so")

SSCN_IMAG, SSCN_REAL = 0, 1
SSCN_C128, SSCN_C64 = 0, 1
PLAN_AUTO, PLAN_SWEEPS, PLAN_FUSED = 0, 1, 2

ERRORS = {0: "SSCN_OK", -1: "SSCN_EINVAL", -2: "SSCN_EOMEGA", -3: "SSCN_EUNSTABLE",
          -4: "SSCN_ENONFINITE", -5: "SSCN_EHIP", -6: "SSCN_ENOMEM"}

# Every symbol include/sscn.h declares.
EXPORTS = ("sscn_init", "sscn_init_state", "sscn_init_state_seed", "sscn_phase_field_seed", "sscn_step", "sscn_prepare_steps", "sscn_observables", "sscn_observables_noalloc",
           "sscn_set_state", "sscn_set_state_device", "sscn_get_state",
           "sscn_set_mode", "sscn_vortex_count", "sscn_profile_step", "sscn_set_plan",
           "sscn_solver_info", "sscn_fused_tile", "sscn_profile_kernel", "sscn_converge", "sscn_get_params", "sscn_batch_init", "sscn_batch_init_state", "sscn_batch_step", "sscn_batch_prepare_steps", "sscn_batch_profile_step",
           "sscn_batch_observables", "sscn_batch_run", "sscn_batch_reset", "sscn_batch_get_state",
           "sscn_batch_set_state_device", "sscn_batch_vortex_count", "sscn_batch_set_plan",
           "sscn_batch_info", "sscn_batch_x_lines", "sscn_batch_destroy", "sscn_embed_state", "sscn_extend_z", "sscn_density", "sscn_resample",
           "sscn_angular_moments",
           "sscn_destroy", "sscn_strerror", "sscn_last_error")


class SSCNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("hx", ctypes.c_double), ("hy", ctypes.c_double),
                ("hz", ctypes.c_double), ("gamma", ctypes.c_double), ("nu", ctypes.c_double),
                ("lam", ctypes.c_double), ("g", ctypes.c_double), ("omega", ctypes.c_double),
                ("dt", ctypes.c_double), ("mode", ctypes.c_int), ("precision", ctypes.c_int)]


class Obs(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double), ("mu", ctypes.c_double), ("energy", ctypes.c_double),
                ("mu_full", ctypes.c_double), ("energy_full", ctypes.c_double),
                ("mu_4th", ctypes.c_double), ("energy_4th", ctypes.c_double),
                ("rms_x", ctypes.c_double), ("rms_y", ctypes.c_double), ("rms_z", ctypes.c_double),
                ("rms_r", ctypes.c_double), ("max_density", ctypes.c_double),
                ("step", ctypes.c_int64), ("sums", ctypes.c_double * 16)]


_lib = None


def lib():
    """Load libsscn.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "paper_1906_06327_amd/build.py (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        L.sscn_init.argtypes = [ctypes.POINTER(Params), vp, vp, ctypes.POINTER(vp)]
        L.sscn_init_state.argtypes = [vp, ctypes.c_int, vp, ctypes.c_double, ctypes.c_double]
        L.sscn_init_state_seed.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                                           ctypes.c_double]
        L.sscn_phase_field_seed.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, vp, vp]
        L.sscn_step.argtypes = [vp, i64]
        L.sscn_prepare_steps.argtypes = [vp, i64]
        L.sscn_observables.argtypes = [vp, ctypes.POINTER(Obs)]
        L.sscn_observables_noalloc.argtypes = [ctypes.POINTER(Params), vp, vp, vp]
        L.sscn_set_state.argtypes = [vp, vp]
        L.sscn_set_state_device.argtypes = [vp]
        L.sscn_get_state.argtypes = [vp, vp]
        L.sscn_set_mode.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
        L.sscn_vortex_count.argtypes = [vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.sscn_solver_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.sscn_fused_tile.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.sscn_set_plan.argtypes = [vp, ctypes.c_int]
        L.sscn_profile_step.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double)]
        L.sscn_profile_kernel.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.sscn_converge.argtypes = [vp, i64, ctypes.c_int, ctypes.c_double, ctypes.c_double, vp,
                                    ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(i64)]
        L.sscn_get_params.argtypes = [vp, ctypes.POINTER(Params)]
        L.sscn_batch_init.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(vp), vp,
                                      ctypes.POINTER(vp)]
        L.sscn_batch_init_state.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_double]
        L.sscn_batch_step.argtypes = [vp, i64]
        L.sscn_batch_prepare_steps.argtypes = [vp, i64]
        L.sscn_batch_profile_step.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double)]
        L.sscn_batch_observables.argtypes = [vp, ctypes.POINTER(Obs)]
        L.sscn_batch_run.argtypes = [vp, i64, ctypes.c_int, ctypes.c_double, ctypes.POINTER(i64)]
        L.sscn_batch_reset.argtypes = [vp]
        L.sscn_batch_get_state.argtypes = [vp, ctypes.c_int, vp]
        L.sscn_batch_set_state_device.argtypes = [vp, ctypes.c_int]
        L.sscn_batch_vortex_count.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_int)]
        L.sscn_batch_set_plan.argtypes = [vp, ctypes.c_int]
        L.sscn_batch_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
        L.sscn_batch_x_lines.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float)]
        L.sscn_density.argtypes = [vp, ctypes.c_int, vp]
        L.sscn_embed_state.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, vp]
        L.sscn_extend_z.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int, vp]
        cd = ctypes.c_double
        L.sscn_resample.argtypes = [vp, ctypes.c_int, ctypes.c_int, cd, cd, vp, ctypes.c_int, ctypes.c_int, cd, cd,
                                    cd, ctypes.c_int, vp]
        L.sscn_angular_moments.argtypes = [vp, ctypes.c_int, ctypes.c_int, cd, cd, ctypes.c_int, ctypes.c_int, vp,
                                           vp]
        L.sscn_batch_destroy.argtypes = [vp]
        L.sscn_batch_destroy.restype = None
        L.sscn_destroy.argtypes = [vp]
        L.sscn_destroy.restype = None
        L.sscn_strerror.argtypes = [ctypes.c_int]
        L.sscn_strerror.restype = ctypes.c_char_p
        L.sscn_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if not hasattr(L, name):
                raise RuntimeError(f"libsscn.so does not export {name}")
        _lib = L
    return _lib


def _check(code):
    if code != 0:
        raise SSCNError(code, lib().sscn_last_error().decode())


def make_params(dim=2, nx=64, ny=64, nz=1, hx=0.1, hy=0.1, hz=0.1, gamma=1.0, nu=1.0,
                lam=1.0, g=0.0, omega=0.0, dt=1e-3, mode=0, precision=0, **_ignored):
    return Params(int(dim), int(nx), int(ny), int(nz if dim == 3 else 1), float(hx), float(hy),
                  float(hz), float(gamma), float(nu), float(lam), float(g), float(omega),
                  float(dt), int(mode), int(precision))


OBS_KEYS = ("norm", "mu", "energy", "mu_full", "energy_full", "mu_4th", "energy_4th", "rms_x", "rms_y", "rms_z",
            "rms_r", "max_density")


def phase_field_seed(seed, ny, nx, stream=None):
    """R(x, y) of sscn_init_state_seed for an ny x nx plane, as a float64
    device tensor (sscn_phase_field_seed)."""
    import torch
    out = torch.empty((ny, nx), dtype=torch.float64, device="cuda")
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().sscn_phase_field_seed(int(seed) & (2**64 - 1), int(nx), int(ny), ctypes.c_void_p(out.data_ptr()),
                                       ctypes.c_void_p(st.cuda_stream)))
    return out


def embed_state(src, dst, stream=None):
    """Centred embedding of the device state tensor `src` into `dst` (same
    spacing, grid sizes differing by an even number of points per axis;
    shapes (ny, nx) or (nz, ny, nx), both complex128 or both complex64):
    the continuation start of Sec. 3.  Asynchronous on `stream` (default:
    the current torch stream)."""
    import torch
    if src.dtype != dst.dtype or src.dtype not in (torch.complex128, torch.complex64):
        raise ValueError("src and dst must both be complex128 or both complex64")
    if src.dim() != dst.dim() or src.dim() not in (2, 3):
        raise ValueError("states are (ny, nx) or (nz, ny, nx)")
    if not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("states must be contiguous")
    shs = (1,) * (3 - src.dim()) + tuple(src.shape)
    shd = (1,) * (3 - dst.dim()) + tuple(dst.shape)
    prec = SSCN_C128 if src.dtype == torch.complex128 else SSCN_C64
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().sscn_embed_state(ctypes.c_void_p(src.data_ptr()), shs[2], shs[1], shs[0],
                                  ctypes.c_void_p(dst.data_ptr()), shd[2], shd[1], shd[0], prec,
                                  ctypes.c_void_p(st.cuda_stream)))


def resample(src, h_src, dst, h, angle=0.0, stream=None):
    """Cubic-convolution interpolation of the 2D device state `src` (ny_s,
    nx_s) with spacings h_src = (hx, hy) onto `dst` (ny, nx) with spacings
    h, sampling src at the destination points rotated by `angle`
    (include/sscn.h, sscn_resample).  Both complex128 or both complex64,
    contiguous.  Asynchronous on `stream` (default: the current torch
    stream)."""
    import torch
    if src.dtype != dst.dtype or src.dtype not in (torch.complex128, torch.complex64):
        raise ValueError("src and dst must both be complex128 or both complex64")
    if src.dim() != 2 or dst.dim() != 2 or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst are contiguous (ny, nx) tensors")
    prec = SSCN_C128 if src.dtype == torch.complex128 else SSCN_C64
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().sscn_resample(ctypes.c_void_p(src.data_ptr()), src.shape[1], src.shape[0], float(h_src[0]),
                               float(h_src[1]), ctypes.c_void_p(dst.data_ptr()), dst.shape[1], dst.shape[0],
                               float(h[0]), float(h[1]), float(angle), prec, ctypes.c_void_p(st.cuda_stream)))


def angular_moments(psi, h, kmax, out=None, stream=None):
    """M_k = hx hy sum |psi|^2 exp(i k phi), k = 0..kmax, of the 2D device
    state `psi` (include/sscn.h, sscn_angular_moments), as a float64 device
    tensor (kmax + 1, 2) of real and imaginary parts (`out` if given).
    Asynchronous on `stream`."""
    import torch
    if psi.dim() != 2 or not psi.is_contiguous() or psi.dtype not in (torch.complex128, torch.complex64):
        raise ValueError("psi is a contiguous complex (ny, nx) tensor")
    if out is None:
        out = torch.empty((kmax + 1, 2), dtype=torch.float64, device=psi.device)
    prec = SSCN_C128 if psi.dtype == torch.complex128 else SSCN_C64
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().sscn_angular_moments(ctypes.c_void_p(psi.data_ptr()), psi.shape[1], psi.shape[0], float(h[0]),
                                      float(h[1]), int(kmax), prec, ctypes.c_void_p(out.data_ptr()),
                                      ctypes.c_void_p(st.cuda_stream)))
    return out


def extend_z(xy, dst, hz, d_z, stream=None):
    """The 3D product start of Eq. (fun): dst[k] = xy * Gaussian(z_k) of
    width d_z, normalised over the interior z points (include/sscn.h,
    sscn_extend_z).  xy: (ny, nx), dst: (nz, ny, nx) contiguous device
    tensors, both complex128 or both complex64.  Asynchronous on `stream`
    (default: the current torch stream)."""
    import torch
    if xy.dtype != dst.dtype or xy.dtype not in (torch.complex128, torch.complex64):
        raise ValueError("xy and dst must both be complex128 or both complex64")
    if xy.dim() != 2 or dst.dim() != 3 or tuple(dst.shape[1:]) != tuple(xy.shape):
        raise ValueError("xy is (ny, nx) and dst (nz, ny, nx)")
    if not (xy.is_contiguous() and dst.is_contiguous()):
        raise ValueError("tensors must be contiguous")
    prec = SSCN_C128 if xy.dtype == torch.complex128 else SSCN_C64
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().sscn_extend_z(ctypes.c_void_p(xy.data_ptr()), xy.shape[1], xy.shape[0],
                               ctypes.c_void_p(dst.data_ptr()), dst.shape[0], float(hz), float(d_z), prec,
                               ctypes.c_void_p(st.cuda_stream)))


def observables_noalloc(params, psi, sums, stream=None):
    """The raw observable sums of the device state tensor `psi` (the
    sscn_obs.sums of sscn_observables) into the float64 device tensor `sums`
    (16 values), without a handle and without allocating: the library's
    static scratch holds the partials (include/sscn.h,
    sscn_observables_noalloc).  Asynchronous on `stream` (default: the
    current torch stream)."""
    import torch
    p = params if isinstance(params, Params) else make_params(**params)
    if sums.dtype != torch.float64 or sums.numel() < 16 or not sums.is_contiguous():
        raise ValueError("sums must be a contiguous float64 device tensor of 16 values")
    if not psi.is_contiguous():
        raise ValueError("psi must be contiguous")
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().sscn_observables_noalloc(ctypes.byref(p), ctypes.c_void_p(psi.data_ptr()),
                                          ctypes.c_void_p(st.cuda_stream), ctypes.c_void_p(sums.data_ptr())))


class Solver:
    """One SSCN problem on the current GPU.

    ``psi`` (a contiguous torch complex128/complex64 CUDA tensor of shape
    (ny, nx) or (nz, ny, nx)) is allocated here unless given; the library
    borrows it.  All work goes to ``stream`` (default: torch's current
    stream)."""

    def __init__(self, params, psi=None, stream=None):
        import torch
        self._torch = torch
        p = params if isinstance(params, Params) else make_params(**params)
        self.params = p
        dtype = torch.complex128 if p.precision == SSCN_C128 else torch.complex64
        shape = (p.nz, p.ny, p.nx) if p.dim == 3 else (p.ny, p.nx)
        if psi is None:
            psi = torch.zeros(shape, dtype=dtype, device="cuda")
        if psi.dtype != dtype or tuple(psi.shape) != shape or not psi.is_contiguous() or not psi.is_cuda:
            raise ValueError("psi must be a contiguous CUDA tensor of the grid shape and precision")
        self.psi = psi
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib().sscn_init(ctypes.byref(p), ctypes.c_void_p(psi.data_ptr()),
                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    @property
    def shape(self):
        p = self.params
        return (p.nz, p.ny, p.nx) if p.dim == 3 else (p.ny, p.nx)

    def init_state(self, kind=1, phase=None, d_xy=1.0, d_z=0.0):
        ph = None
        if phase is not None:
            ph = np.ascontiguousarray(phase, dtype=np.float64)
            if ph.shape != (self.params.ny, self.params.nx):
                raise ValueError("phase must have shape (ny, nx)")
        _check(lib().sscn_init_state(self._h, int(kind), ph.ctypes.data if ph is not None else None,
                                     float(d_xy), float(d_z)))

    def init_state_seed(self, kind=1, seed=13, d_xy=1.0, d_z=0.0, random_phase=True):
        """Eq. (fun) with R(x, y) from the device's counter-based generator
        (sscn_init_state_seed); random_phase=False: no random phase."""
        _check(lib().sscn_init_state_seed(self._h, int(kind), 1 if random_phase else 0, int(seed) & (2**64 - 1),
                                          float(d_xy), float(d_z)))

    def step(self, n=1):
        _check(lib().sscn_step(self._h, int(n)))

    def prepare_steps(self, n):
        """Plan choice and graph capture of a later step(n), without stepping."""
        _check(lib().sscn_prepare_steps(self._h, int(n)))

    def observables(self, raise_nonfinite=True):
        o = Obs()
        code = lib().sscn_observables(self._h, ctypes.byref(o))
        if code != 0 and (raise_nonfinite or code != -4):
            _check(code)
        d = {k: getattr(o, k) for k in OBS_KEYS}
        d["step"] = int(o.step)
        d["sums"] = np.array(list(o.sums))
        return d

    def set_state(self, host):
        dtype = np.complex128 if self.params.precision == SSCN_C128 else np.complex64
        a = np.ascontiguousarray(host, dtype=dtype)
        if a.shape != self.shape:
            raise ValueError(f"state shape {a.shape} != {self.shape}")
        _check(lib().sscn_set_state(self._h, a.ctypes.data))

    def set_state_device(self):
        _check(lib().sscn_set_state_device(self._h))

    def get_state(self):
        dtype = np.complex128 if self.params.precision == SSCN_C128 else np.complex64
        out = np.empty(self.shape, dtype=dtype)
        _check(lib().sscn_get_state(self._h, out.ctypes.data))
        return out

    def set_mode(self, mode, precision=None):
        torch = self._torch
        if precision is None:
            precision = self.params.precision
        new = None
        if precision != self.params.precision:
            dtype = torch.complex128 if precision == SSCN_C128 else torch.complex64
            new = torch.empty(self.shape, dtype=dtype, device=self.psi.device)
        _check(lib().sscn_set_mode(self._h, int(mode), int(precision),
                                   ctypes.c_void_p(new.data_ptr()) if new is not None else None))
        self.params.mode = int(mode)
        self.params.precision = int(precision)
        if new is not None:
            self.psi = new

    def converge(self, max_steps, check_every=100, tol=1e-8, switch_tol=2e-6):
        """Run imaginary time to |dmu| < tol at two consecutive checks with an
        unchanged vortex count; complex64 runs switch to complex128 at their
        plateau (into a complex128 tensor allocated here, which becomes
        self.psi).  Returns (steps, converged); self.switch_step is the step
        of the upcast (-1 if none)."""
        torch = self._torch
        new = None
        if self.params.precision == SSCN_C64:
            new = torch.empty(self.shape, dtype=torch.complex128, device=self.psi.device)
        steps, ok, sw = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int64()
        try:
            _check(lib().sscn_converge(self._h, int(max_steps), int(check_every), float(tol),
                                       float(switch_tol),
                                       ctypes.c_void_p(new.data_ptr()) if new is not None else None,
                                       ctypes.byref(steps), ctypes.byref(ok), ctypes.byref(sw)))
        finally:
            # the handle borrows `new` from the upcast on, even when a later
            # call of the run failed: keep the tensor alive with it
            p = Params()
            if lib().sscn_get_params(self._h, ctypes.byref(p)) == 0:
                if new is not None and p.precision == SSCN_C128:
                    self.psi = new
                self.params = p
        self.switch_step = int(sw.value)
        return int(steps.value), bool(ok.value)

    def vortex_count(self, density_frac=0.05, box=3):
        c = ctypes.c_int()
        _check(lib().sscn_vortex_count(self._h, float(density_frac), int(box), ctypes.byref(c)))
        return int(c.value)

    DENSITY_KINDS = {"full": 0, "xy": 1, "x": 2, "y": 3, "z": 4, "cut_x": 5, "cut_y": 6, "cut_z": 7}

    def density(self, kind="full"):
        """A density profile (sscn_density) as a float64 device tensor:
        'full' (the state's shape), 'xy' (ny, nx), 'x', 'y', 'z' (integrals
        over the other axes), 'cut_x', 'cut_y', 'cut_z' (through the
        centre)."""
        torch = self._torch
        k = self.DENSITY_KINDS[kind]
        p = self.params
        nz = p.nz if p.dim == 3 else 1
        shape = {0: self.shape, 1: (p.ny, p.nx), 2: (p.nx,), 3: (p.ny,), 4: (nz,),
                 5: (p.nx,), 6: (p.ny,), 7: (nz,)}[k]
        out = torch.empty(shape, dtype=torch.float64, device=self.psi.device)
        _check(lib().sscn_density(self._h, k, ctypes.c_void_p(out.data_ptr())))
        return out

    def profile_step(self, n):
        """Advance n steps, each kernel launched alone between HIP events;
        returns average milliseconds of the x, y, z sweeps and of a step."""
        ms = (ctypes.c_double * 4)()
        _check(lib().sscn_profile_step(self._h, int(n), ms))
        return {"x": ms[0], "y": ms[1], "z": ms[2], "step": ms[3]}

    def profile_kernel(self, which=0, n=200):
        """Average ms of kernel `which` (0 fused step or x-sweep, 1 y, 2 z)
        over n back-to-back launches (HIP events on the solver's stream)."""
        ms = ctypes.c_double()
        _check(lib().sscn_profile_kernel(self._h, int(which), int(n), ctypes.byref(ms)))
        return ms.value

    def set_plan(self, plan):
        _check(lib().sscn_set_plan(self._h, int(plan)))

    def solver_info(self):
        w = (ctypes.c_int * 3)()
        s = (ctypes.c_int * 3)()
        pl = ctypes.c_int()
        xl = ctypes.c_int()
        _check(lib().sscn_solver_info(self._h, w, s, ctypes.byref(pl), ctypes.byref(xl)))
        tr, tc = ctypes.c_int(), ctypes.c_int()
        _check(lib().sscn_fused_tile(self._h, ctypes.byref(tr), ctypes.byref(tc)))
        return {"window": list(w), "segment": list(s), "plan": int(pl.value), "x_lines": int(xl.value),
                "fused_tile": [int(tr.value), int(tc.value)]}

    def close(self):
        if getattr(self, "_h", None):
            lib().sscn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """n instances (all 2D or all 3D) advanced together (include/sscn.h,
    sscn_batch_*).  State tensors are allocated here (torch, one per
    instance, shape (ny, nx) or (nz, ny, nx)) and borrowed by the library."""

    def __init__(self, params_list, stream=None):
        import torch
        self._torch = torch
        ps = [p if isinstance(p, Params) else make_params(**p) for p in params_list]
        self.params = ps
        n = len(ps)
        arr = (Params * n)(*ps)
        dtype = torch.complex128 if ps[0].precision == SSCN_C128 else torch.complex64
        self.psi = [torch.zeros((p.nz, p.ny, p.nx) if p.dim == 3 else (p.ny, p.nx), dtype=dtype, device="cuda")
                    for p in ps]
        ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.psi])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib().sscn_batch_init(arr, n, ptrs, ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(h)))
        self._h = h
        self.n = n

    def init_state(self, k, kind=1, phase=None, d_xy=1.0):
        ph = None
        if phase is not None:
            ph = np.ascontiguousarray(phase, dtype=np.float64)
            if ph.shape != (self.params[k].ny, self.params[k].nx):
                raise ValueError("phase must have shape (ny, nx)")
        _check(lib().sscn_batch_init_state(self._h, int(k), int(kind),
                                           ph.ctypes.data if ph is not None else None, float(d_xy)))

    def step(self, n=1):
        _check(lib().sscn_batch_step(self._h, int(n)))

    def prepare_steps(self, n):
        """Plan choice and graph capture of a later step(n), without stepping."""
        _check(lib().sscn_batch_prepare_steps(self._h, int(n)))

    def profile_step(self, n):
        """Advance n steps launched one by one with HIP events around every
        kernel; average ms of the x-sweep and y-sweep (sweep plan) or of the
        fused step, and of a whole step."""
        ms = (ctypes.c_double * 4)()
        _check(lib().sscn_batch_profile_step(self._h, int(n), ms))
        if self.info()["plan"] == PLAN_SWEEPS:
            out = {"x": ms[0], "y": ms[1], "step": ms[3]}
            if self.params[0].dim == 3:
                out["z"] = ms[2]
            return out
        return {"fused": ms[0], "step": ms[3]}

    def run(self, max_steps, check_every=100, tol=1e-8):
        out = (ctypes.c_int64 * self.n)()
        _check(lib().sscn_batch_run(self._h, int(max_steps), int(check_every), float(tol), out))
        return [int(v) for v in out]

    def reset(self):
        _check(lib().sscn_batch_reset(self._h))

    def observables(self):
        out = (Obs * self.n)()
        _check(lib().sscn_batch_observables(self._h, out))
        res = []
        for o in out:
            d = {k: getattr(o, k) for k in OBS_KEYS}
            d["step"] = int(o.step)
            res.append(d)
        return res

    def get_state(self, k):
        p = self.params[k]
        dtype = np.complex128 if p.precision == SSCN_C128 else np.complex64
        out = np.empty((p.nz, p.ny, p.nx) if p.dim == 3 else (p.ny, p.nx), dtype=dtype)
        _check(lib().sscn_batch_get_state(self._h, int(k), out.ctypes.data))
        return out

    def set_plan(self, plan):
        _check(lib().sscn_batch_set_plan(self._h, int(plan)))

    def info(self):
        pl, w = ctypes.c_int(), ctypes.c_int()
        _check(lib().sscn_batch_info(self._h, ctypes.byref(pl), ctypes.byref(w)))
        xo, xt = ctypes.c_int(), (ctypes.c_float * 2)()
        _check(lib().sscn_batch_x_lines(self._h, ctypes.byref(xo), xt))
        return {"plan": int(pl.value), "window": int(w.value), "x_lines_option": int(xo.value),
                "x_lines_tune_ms": [float(xt[0]), float(xt[1])]}

    def set_state_device(self, k):
        """Instance k's tensor self.psi[k] was written in place: zero its
        walls and normalise it."""
        _check(lib().sscn_batch_set_state_device(self._h, int(k)))

    def vortex_count(self, k, density_frac=0.05, box=3):
        c = ctypes.c_int()
        _check(lib().sscn_batch_vortex_count(self._h, int(k), float(density_frac), int(box), ctypes.byref(c)))
        return c.value

    def close(self):
        if getattr(self, "_h", None):
            lib().sscn_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
