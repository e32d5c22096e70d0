"""Dense brute-force forms used to pin the oracle (test helper, numpy only).

These build the line Hamiltonians of Eqs. (eq2)/(eq3) as dense matrices and
apply textbook Crank-Nicolson with numpy's LU solve.  They do not use the
tridiagonal coefficients A-, A0, A+ or b of Eqs. (eqD.11)/(eq5) or any Thomas
algorithm, so agreement with the oracle pins those.
"""
import numpy as np


def coords(n, h):
    return -0.5 * n * h + h * np.arange(n)


def line_hamiltonian(n, h, axis, transverse, omega):
    """Dense H on the n-1 unknowns of a line.

    x-line at y:  H2 = -1/2 d2/dx2 - i Omega y d/dx   (Eq. (eq2))
    y-line at x:  H3 = -1/2 d2/dy2 + i Omega x d/dy   (Eq. (eq3))
    z-line:       -1/2 d2/dz2
    with the 3-point second difference and the central first difference,
    Dirichlet zero at both ends."""
    m = n - 1
    lap = (np.diag(-2.0 * np.ones(m)) + np.diag(np.ones(m - 1), 1)
           + np.diag(np.ones(m - 1), -1)) / (h * h)
    dif = (np.diag(np.ones(m - 1), 1) - np.diag(np.ones(m - 1), -1)) / (2.0 * h)
    H = -0.5 * lap.astype(np.complex128)
    if axis == 0:
        H = H - 1j * omega * transverse * dif
    elif axis == 1:
        H = H + 1j * omega * transverse * dif
    return H


def cn_matrix(H, dt, mode):
    """Textbook Crank-Nicolson propagator over dt.

    real time (mode 1):      (1 + i dt H / 2) psi' = (1 - i dt H / 2) psi
    imaginary time (mode 0): (1 + dt H / 2) psi'   = (1 - dt H / 2) psi"""
    I = np.eye(H.shape[0], dtype=np.complex128)
    K = (1j * dt / 2.0) * H if mode == 1 else (dt / 2.0) * H
    return np.linalg.solve(I + K, I - K)


def apply_axis(psi, p, axis):
    """Apply the dense CN propagator along `axis` to every line of psi."""
    out = np.array(psi, dtype=np.complex128, copy=True)
    dim = p.dim
    hs = (p.hx, p.hy, p.hz)
    ns = (p.nx, p.ny, p.nz)
    n, h = ns[axis], hs[axis]
    npax = (dim - 1) - axis  # numpy axis of the grid axis
    moved = np.moveaxis(out, npax, -1)  # view, lines along last axis
    it = np.ndindex(moved.shape[:-1])
    for idx in it:
        if axis == 0:
            transverse = coords(p.ny, p.hy)[idx[-1]]
        elif axis == 1:
            transverse = coords(p.nx, p.hx)[idx[-1]]
        else:
            transverse = 0.0
        C = cn_matrix(line_hamiltonian(n, h, axis, transverse, p.omega), p.dt, p.mode)
        line = moved[idx]
        new = np.zeros_like(line)
        new[1:] = C @ line[1:]
        moved[idx] = new
    return out


def potential_grid(p):
    x = coords(p.nx, p.hx)
    y = coords(p.ny, p.hy)
    if p.dim == 2:
        Y, X = np.meshgrid(y, x, indexing="ij")
        return 0.5 * (p.gamma ** 2 * X ** 2 + p.nu ** 2 * Y ** 2)
    z = coords(p.nz, p.hz)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return 0.5 * (p.gamma ** 2 * X ** 2 + p.nu ** 2 * Y ** 2 + p.lam ** 2 * Z ** 2)


def dense_step(p, psi):
    """One split step by brute force: nonlinear/potential factor, then the
    dense CN propagators along x, y (and z), then renormalisation in
    imaginary time."""
    V = potential_grid(p)
    w = V + p.g * np.abs(psi) ** 2
    if p.mode == 1:
        out = np.exp(-1j * p.dt * w) * psi
    else:
        out = np.exp(-p.dt * w) * psi
    out = apply_axis(out, p, 0)
    out = apply_axis(out, p, 1)
    if p.dim == 3:
        out = apply_axis(out, p, 2)
    if p.mode == 0:
        dv = p.hx * p.hy * (p.hz if p.dim == 3 else 1.0)
        out = out / np.sqrt(dv * np.sum(np.abs(out) ** 2))
    return out
