// Host-only parts of the library: Chebyshev and Fermi coefficients, the
// sample average, the DOS, moment and response transforms, and the patch
// planner's C entry points.  Nothing here touches the GPU, so these sources
// (tbpm_host.cpp, tbpm_bessel.cpp, tbpm_patch.cpp) also build with a plain
// C++ compiler, e.g. for a sanitizer build of the host logic.
#pragma once

#include <cstddef>
#include <vector>

#include "../../include/tbpm.h"

namespace tbpm {

// Bessel / coefficients (tbpm_bessel.cpp)
int chebyshev_coefficients(double tau, double eps, int max_terms, double *coeff);
// j[0..mmax] = J_m(x) for x > 0 (Miller's backward recurrence)
bool bessel_all(double x, int mmax, std::vector<double> &j);
// Chebyshev coefficients a_m of the Fermi function f(rescale x) on [-1, 1],
// truncated after the last |a_m| >= eps (tbpm_host.cpp); false if they do
// not converge
bool fermi_coefficients(double rescale, double mu, double kT, double eps, std::vector<double> &a);
// Sample average over the R vectors of per-vector correlation rows:
// mean[k] = (1/R) sum_{r=0}^{R-1} rows[r][k], k < nt1, complex interleaved;
// rows is [R][nt1] when row_major, else [nt1][R].  Summed in the order
// r = 0, 1, ..., R-1 in FP64, so the result does not depend on the blocking.
void sample_mean(const double *rows, size_t R, size_t nt1, bool row_major, double *mean);

}  // namespace tbpm
