// Host-only parts of the library: Chebyshev and Fermi coefficients, the
// sample average, the DOS, moment and response transforms, and the patch
// planner's C entry points.  Nothing here touches the GPU, so these sources
// (tbpm_host.cpp, tbpm_bessel.cpp, tbpm_patch.cpp) also build with a plain
// C++ compiler, e.g. for a sanitizer build of the host logic.
#pragma once

#include <cstddef>
#include <cstdint>
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

// Value table of a tight-binding H: the hoppings of a supercell are copies of
// the few hoppings of its primitive cell, so the off-diagonal entries often
// take only a handful of distinct values.  A stored H may then hold a table
// of at most 255 values and one byte per entry (index 255: the row's own
// diagonal value, kept in a per-row array when the on-site energies are
// many, e.g. under Anderson disorder).  Values are compared bit for bit in
// the stored precision (complex128, or each part rounded to float for
// complex64), so the table gives back exactly the values the entries hold.
struct ValueTable {
    // sorted keys, two words per value: the bit patterns of the real and the
    // imaginary part (complex64: the float bit patterns, zero-extended);
    // keys[0], keys[1] = 0, 0: +0 is always entry 0 (ELL padding)
    std::vector<uint64_t> keys;
    bool diag = false;          // diagonal entries take index 255 and a per-row value
    bool diag_real = false;     // ... whose imaginary parts are all +0: the real part alone is kept
};
// Plans the table from a host CSR (val complex128 interleaved).  False when
// the off-diagonal entries take more than 254 distinct nonzero values, or
// when the diagonal needs the per-row array but a row has two nonzero
// diagonal entries.
bool plan_value_table(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val, int dtype,
                      ValueTable &vt);

}  // namespace tbpm
