// Plain parameter structs shared by the host setup (sscn_setup.cpp, no HIP)
// and the kernels (sscn_device.hpp).
#pragma once

namespace sscn {

// Per-axis Crank-Nicolson coefficients (FP64, from the host):
//   A0 = 1 + k0, k0 = i tau/(2h^2),  A+- = u +- q rot,  u = -i tau/(4h^2),
//   q = tau/(4h); rot = Omega y_j (x-lines), -Omega x_i (y-lines), 0 (z).
struct AxisCoef {
    double a0r, a0i, k0r, k0i, ur, ui, qr, qi;
};

struct StepArgs {
    int dim, nx, ny, nz;
    double hx, hy, hz;
    double x0, y0, z0;          // first stored coordinate, -n h / 2
    double vx, vy, vz;          // 1/2 gamma^2, 1/2 nu^2, 1/2 lambda^2
    double g, omega, dt, dV;
    AxisCoef ax[3];
};

}  // namespace sscn
