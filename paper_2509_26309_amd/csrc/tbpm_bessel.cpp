// Chebyshev coefficients of the time-evolution operator.
//
// exp(-i tau x) = J_0(tau) + 2 sum_{m>=1} (-i)^m J_m(tau) T_m(x)   (Jacobi-Anger),
// so c_0 = J_0(tau) and c_m = 2 (-i)^m J_m(tau): the imaginary factor of the
// time step sits in the coefficients and the recurrence itself stays real
// (TBPLaS 2.0, "Migration to C++").
//
// J_m(tau) for all m at once by Miller's backward recurrence
// (Abramowitz & Stegun 9.12; J. C. P. Miller, 1952): starting far above the
// wanted orders from (0, tiny), J_{m-1} = (2m / tau) J_m - J_{m+1} runs in the
// stable direction; the result is normalised with J_0 + 2 sum_k J_{2k} = 1.
#include <cmath>
#include <vector>

#include "tbpm_host.h"

namespace tbpm {

// j[0..mmax] = J_m(x), x > 0
bool bessel_all(double x, int mmax, std::vector<double> &j)
{
    if (!(x > 0.0) || mmax < 0)
        return false;
    // start well above both the wanted order and the turning point m = x
    int start = mmax + 20 + (int)std::sqrt(40.0 * (mmax + 1));
    if (start < (int)x + 40)
        start = (int)x + 40;
    if (start & 1)
        ++start;
    std::vector<double> t((size_t)start + 2, 0.0);
    double jp1 = 0.0, jm = 1e-300;
    t[(size_t)start] = jm;
    for (int m = start; m >= 1; --m) {
        const double jm1 = (2.0 * m / x) * jm - jp1;
        jp1 = jm;
        jm = jm1;
        t[(size_t)m - 1] = jm;
        if (std::fabs(jm) > 1e250) {           // rescale everything computed so far
            for (int k = m - 1; k <= start; ++k)
                t[(size_t)k] *= 1e-250;
            jm *= 1e-250;
            jp1 *= 1e-250;
        }
    }
    double norm = t[0];
    for (int k = 2; k <= start; k += 2)
        norm += 2.0 * t[(size_t)k];
    j.assign((size_t)mmax + 1, 0.0);
    for (int m = 0; m <= mmax; ++m)
        j[(size_t)m] = t[(size_t)m] / norm;
    return true;
}

// Writes c_m (interleaved complex) for m < M into coeff[2*max_terms] and
// returns M = first m > tau with |J_m(tau)| < eps; -1 when M > max_terms or
// the arguments are invalid.
int chebyshev_coefficients(double tau, double eps, int max_terms, double *coeff)
{
    if (!(tau > 0.0) || !(eps > 0.0) || max_terms < 1 || !std::isfinite(tau))
        return -1;
    int mmax = (int)std::ceil(tau) + 30 + (int)(10.0 * std::cbrt(tau));
    std::vector<double> j;
    for (int attempt = 0; attempt < 8; ++attempt, mmax *= 2) {
        if (!bessel_all(tau, mmax, j))
            return -1;
        int M = -1;
        for (int m = 0; m <= mmax; ++m) {
            if ((double)m > tau && std::fabs(j[(size_t)m]) < eps) {
                M = m;
                break;
            }
        }
        if (M < 0)
            continue;
        if (M > max_terms)
            return -1;
        for (int m = 0; m < M; ++m) {
            const double a = (m == 0 ? 1.0 : 2.0) * j[(size_t)m];
            // (-i)^m = 1, -i, -1, i for m mod 4 = 0, 1, 2, 3
            double re = 0.0, im = 0.0;
            switch (m & 3) {
            case 0: re = a; break;
            case 1: im = -a; break;
            case 2: re = -a; break;
            default: im = a; break;
            }
            coeff[2 * m] = re;
            coeff[2 * m + 1] = im;
        }
        return M;
    }
    return -1;
}

}  // namespace tbpm
