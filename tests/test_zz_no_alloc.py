"""The allocation-free observables entry point against sscn_observables.

sscn_observables_noalloc (for callers that cannot allocate device memory)
writes the raw observable sums of a state into a caller-owned device
buffer, its partial sums living in the library's static scratch.  Its
output must equal the handle-based sscn_observables' sums on the same state
(same kernels, same reduction order: the same bits), on two calls in a
row, the second on a smaller grid, in both precisions and in 3D."""
import numpy as np
import pytest

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


def cfg(nx, ny, nz=1, prec=0):
    c = dict(dim=2 if nz == 1 else 3, nx=nx, ny=ny, nz=nz, hx=0.11, hy=0.1, hz=0.2, gamma=1.0, nu=1.1, lam=2.0,
             g=80.0, omega=0.6, dt=1e-3, mode=0, precision=prec)
    return c


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dim", [2, 3])
def test_noalloc_observables_equal_handle_observables(P, prec, dim):
    import torch
    print(f"[gpu-noalloc] prec={prec} dim={dim}", flush=True)
    shapes = [(300, 260, 1), (90, 70, 1)] if dim == 2 else [(96, 80, 40), (40, 36, 20)]
    sums = torch.full((16,), float("nan"), dtype=torch.float64, device="cuda")
    for k, (nx, ny, nz) in enumerate(shapes):  # the second call on a smaller grid
        c = cfg(nx, ny, nz, prec)
        s = P.Solver(W.solver_params(c))
        s.init_state(1, W.phase_field(40 + k, ny, nx), 1.0)
        s.step(7)
        ref = s.observables()["sums"]
        torch.cuda.synchronize()
        P.observables_noalloc(W.solver_params(c), s.psi, sums)
        torch.cuda.synchronize()
        got = sums.cpu().numpy()
        assert np.array_equal(got, ref), (k, got - ref)
        s.close()
