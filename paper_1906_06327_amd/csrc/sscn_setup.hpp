// Host-side setup of the solver (sscn_setup.cpp): plain C++ without HIP, so
// that it builds on its own (with the sanitizers, in the tests) as well as
// into libsscn.so.
#pragma once

#include "sscn.h"
#include "sscn_types.hpp"

#include <complex>
#include <string>
#include <vector>

namespace sscn {

// Supported window sizes (template instantiations of the sweep kernels).
const int kWindows[] = {4, 6, 8, 10, 12, 13, 14, 16, 20, 24, 32};

// Record msg as the calling thread's last error (sscn_last_error) and
// return code.
int fail(int code, const std::string &msg);
const char *last_error();

// Smallest window W whose truncation error bound is at most tol for a
// strictly diagonally dominant tridiagonal Toeplitz system with |A-| <= ab,
// |A0| = bb, |A+| <= cb; -1 if not diagonally dominant.
int window_rows(double ab, double bb, double cb, double tol);
// 0 for valid parameters, else SSCN_EINVAL or SSCN_EOMEGA (message via fail).
int validate(const sscn_params &p);
// Crank-Nicolson coefficients of one axis and its window (0: the exact
// whole-line path); SSCN_EUNSTABLE if the line systems are not diagonally
// dominant.
int axis_setup(const sscn_params &p, int axis, AxisCoef &c, int &W);
// Grid geometry and physical constants (everything of StepArgs but ax[]).
void fill_args(const sscn_params &p, StepArgs &a);
// Fixed point c* = A+ / (A0 - A- c*) of the Thomas recurrence.
std::complex<double> pivot_fixed_point(std::complex<double> A0, std::complex<double> Am, std::complex<double> Ap);
// Pivot table of axis ax with window W (rows of W + 2 values per line type).
void pivot_table(const sscn_params &p, const StepArgs &a, int ax, int W, std::vector<std::complex<double>> &t);

}  // namespace sscn
