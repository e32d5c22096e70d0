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

// Staged x-line layout of the x-sweeps (segments of S outputs, window halo
// W).  Point u of a line sits at LDS entry x_row_index(u + x_row_off(S, W),
// S): one padding entry after every S points, so that the threads of
// consecutive segments hit different banks.  The row covers u = -off ..
// nx - 1 + S + W, where off = x_row_off(S, W) >= W + 1 is a multiple of S;
// the entries outside the unknowns 1..nx-1 hold zeros, so every window of a
// segment (points s - W - 1 .. s + S + W) reads the row at constant offsets
// from the segment's base entry without a bounds test.
constexpr int x_row_off(int S, int W) { return S * ((W + S) / S); }
constexpr int x_row_index(int U, int S) { return U + U / S; }
constexpr int x_row_len(int nx, int S, int W) { return x_row_index(nx + S + W + x_row_off(S, W), S) + 1; }

}  // namespace sscn
