// Host-only functions of the C ABI (see tbpm_host.h): no GPU work.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#include "tbpm_host.h"
#include "tbpm_patch.h"

namespace tbpm {

void sample_mean(const double *rows, size_t R, size_t nt1, bool row_major, double *mean)
{
    for (size_t k2 = 0; k2 < nt1; ++k2) {
        double re = 0.0, im = 0.0;
        for (size_t r = 0; r < R; ++r) {
            const size_t at = row_major ? r * nt1 + k2 : k2 * R + r;
            re += rows[2 * at];
            im += rows[2 * at + 1];
        }
        mean[2 * k2] = re / (double)R;
        mean[2 * k2 + 1] = im / (double)R;
    }
}

// Key of a value in the stored precision: the bit patterns of its parts.
static inline void value_key(const double *v, int dtype, uint64_t &re, uint64_t &im)
{
    if (dtype == TBPM_C64) {
        const float fr = (float)v[0], fi = (float)v[1];
        uint32_t a, b;
        std::memcpy(&a, &fr, 4);
        std::memcpy(&b, &fi, 4);
        re = a;
        im = b;
    } else {
        std::memcpy(&re, &v[0], 8);
        std::memcpy(&im, &v[1], 8);
    }
}

namespace {
// a small set of keys with a cache of the last hit (runs of equal hoppings)
struct KeySet {
    std::vector<uint64_t> k;    // pairs
    size_t cap, last = 0;
    bool over = false;
    explicit KeySet(size_t c) : cap(c) {}
    void add(uint64_t re, uint64_t im)
    {
        if (over)
            return;
        if (!k.empty() && k[2 * last] == re && k[2 * last + 1] == im)
            return;
        for (size_t i = 0; i < k.size() / 2; ++i)
            if (k[2 * i] == re && k[2 * i + 1] == im) {
                last = i;
                return;
            }
        if (k.size() / 2 >= cap) {
            over = true;
            return;
        }
        k.push_back(re);
        k.push_back(im);
        last = k.size() / 2 - 1;
    }
};
}  // namespace

bool plan_value_table(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val, int dtype,
                      ValueTable &vt)
{
    vt.keys.clear();
    vt.diag = false;
    KeySet off(254), dg(254);
    bool two_diag = false, dg_real = true;
    for (int64_t i = 0; i < n; ++i) {
        int nd = 0;
        for (int64_t j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
            uint64_t re, im;
            value_key(val + 2 * j, dtype, re, im);
            if (re == 0 && im == 0)
                continue;                       // +0 is entry 0
            if (col[j] == i) {
                ++nd;
                dg.add(re, im);
                dg_real &= im == 0;
            } else {
                off.add(re, im);
                if (off.over)
                    return false;
            }
        }
        two_diag |= nd > 1;
    }
    std::vector<std::pair<uint64_t, uint64_t>> all;
    for (size_t q = 0; q < off.k.size() / 2; ++q)
        all.emplace_back(off.k[2 * q], off.k[2 * q + 1]);
    if (!dg.over) {
        for (size_t q = 0; q < dg.k.size() / 2; ++q)
            all.emplace_back(dg.k[2 * q], dg.k[2 * q + 1]);
    }
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    if (dg.over || all.size() > 254) {
        // the diagonal goes to the per-row array: the table holds the rest
        if (two_diag)
            return false;
        vt.diag = true;
        vt.diag_real = dg_real;
        all.clear();
        for (size_t q = 0; q < off.k.size() / 2; ++q)
            all.emplace_back(off.k[2 * q], off.k[2 * q + 1]);
        std::sort(all.begin(), all.end());
    }
    vt.keys.reserve(2 * (all.size() + 1));
    vt.keys.push_back(0);
    vt.keys.push_back(0);
    for (const auto &p : all) {
        vt.keys.push_back(p.first);
        vt.keys.push_back(p.second);
    }
    return vt.keys.size() / 2 <= 255;
}

// In-place radix-2 FFT (length a power of two), forward sign e^{-2 pi i jk/N}.
static void fft(std::vector<std::complex<double>> &a)
{
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1)
            j ^= bit;
        j ^= bit;
        if (i < j)
            std::swap(a[i], a[j]);
    }
    const double pi = 3.141592653589793238462643383279;
    for (size_t len = 2; len <= n; len <<= 1) {
        const double ang = -2.0 * pi / (double)len;
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const std::complex<double> w(std::cos(ang * (double)k), std::sin(ang * (double)k));
                const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
    }
}

// a_m = (2 - delta_m0)/K sum_k f(rho cos theta_k) cos(m theta_k), theta_k = pi (k + 1/2)/K,
// i.e. a DCT-II of the samples, taken with one FFT of the even extension (length 2K);
// K doubles until the coefficients fall below eps well before m = K/4.
bool fermi_coefficients(double rescale, double mu, double kT, double eps, std::vector<double> &a)
{
    if (!(rescale > 0.0) || !(kT > 0.0) || !(eps > 0.0) || !std::isfinite(mu))
        return false;
    const double pi = 3.141592653589793238462643383279;
    for (size_t K = 1024; K <= ((size_t)1 << 21); K <<= 1) {
        std::vector<std::complex<double>> y(2 * K);
        for (size_t k = 0; k < K; ++k) {
            const double e = rescale * std::cos(pi * ((double)k + 0.5) / (double)K);
            const double x = (e - mu) / kT;
            const double f = x > 0.0 ? std::exp(-x) / (1.0 + std::exp(-x)) : 1.0 / (1.0 + std::exp(x));
            y[k] = f;
            y[2 * K - 1 - k] = f;
        }
        fft(y);
        const size_t mmax = K / 4;
        a.assign(mmax, 0.0);
        long last = -1;
        for (size_t m = 0; m < mmax; ++m) {
            const double ph = -pi * (double)m / (2.0 * (double)K);
            const double dct = 0.5 * (y[m] * std::complex<double>(std::cos(ph), std::sin(ph))).real();
            a[m] = (m == 0 ? 1.0 : 2.0) * dct / (double)K;
            if (std::fabs(a[m]) >= eps)
                last = (long)m;
        }
        if (last + 1 < (long)mmax / 2) {
            a.resize((size_t)std::max(last + 1, 1L));
            return true;
        }
    }
    return false;
}

}  // namespace tbpm

using namespace tbpm;

extern "C" {

const char *tbpm_status_string(tbpm_status s)
{
    switch (s) {
    case TBPM_OK: return "ok";
    case TBPM_PENDING: return "pending";
    case TBPM_ERR_ARG: return "invalid argument";
    case TBPM_ERR_CSR: return "malformed or non-Hermitian CSR";
    case TBPM_ERR_RESCALE: return "rescale below the Gershgorin bound";
    case TBPM_ERR_TOO_LARGE: return "request larger than the memory budget";
    case TBPM_ERR_OOM: return "out of device memory";
    case TBPM_ERR_DIVERGED: return "norm drift beyond tolerance";
    case TBPM_ERR_HIP: return "HIP runtime error";
    case TBPM_ERR_CANCELLED: return "cancelled";
    case TBPM_ERR_UNKNOWN: return "unknown ticket";
    default: return "unknown status";
    }
}

tbpm_status tbpm_coefficients(double tau, double eps, int32_t max_terms, double *coeff, int32_t *num_terms)
{
    if (!coeff || !num_terms || max_terms < 1)
        return TBPM_ERR_ARG;
    const int m = chebyshev_coefficients(tau, eps, max_terms, coeff);
    if (m < 0)
        return TBPM_ERR_ARG;
    *num_terms = m;
    return TBPM_OK;
}

tbpm_status tbpm_sample_mean(const double *rows, int32_t num_rows, int32_t len, double *mean)
{
    if (!rows || !mean || num_rows < 1 || len < 0)
        return TBPM_ERR_ARG;
    sample_mean(rows, (size_t)num_rows, (size_t)len, true, mean);
    return TBPM_OK;
}

tbpm_status tbpm_dos(const double *corr, int32_t num_time_steps, double rescale, int32_t window, double *energies,
                     double *dos)
{
    if (!corr || !energies || !dos || num_time_steps < 1 || !(rescale > 0.0) || (window != 0 && window != 1))
        return TBPM_ERR_ARG;
    const double pi = 3.141592653589793238462643383279;
    const int nt = num_time_steps;
    const double dt = pi / rescale;
    // weights and the time grid once; then one cosine/sine pair per (E, t)
    std::vector<double> w((size_t)nt + 1);
    for (int k = 0; k <= nt; ++k)
        w[(size_t)k] = window ? 0.5 * (1.0 + std::cos(pi * k / nt)) : 1.0;
    for (int j = 0; j < 2 * nt; ++j) {
        const double e = -rescale + (double)j * rescale / nt;
        double acc = w[0] * corr[0];
        for (int k = 1; k <= nt; ++k) {
            const double ph = e * k * dt;
            acc += 2.0 * w[(size_t)k] * (corr[2 * k] * std::cos(ph) - corr[2 * k + 1] * std::sin(ph));
        }
        energies[j] = e;
        dos[j] = dt / (2.0 * pi) * acc;
    }
    return TBPM_OK;
}

tbpm_status tbpm_fermi_coefficients(double rescale, double mu, double kT, double eps, int32_t max_terms,
                                    double *coeff, int32_t *num_terms)
{
    if (!coeff || !num_terms || max_terms < 1)
        return TBPM_ERR_ARG;
    std::vector<double> a;
    if (!fermi_coefficients(rescale, mu, kT, eps, a) || (int32_t)a.size() > max_terms)
        return TBPM_ERR_ARG;
    std::copy(a.begin(), a.end(), coeff);
    *num_terms = (int32_t)a.size();
    return TBPM_OK;
}

tbpm_status tbpm_ac_conductivity(const double *corr, int32_t num_time_steps, double rescale, double kT,
                                 double area_per_orbital, int32_t num_omegas, const double *omegas, double *sigma)
{
    if (!corr || !omegas || !sigma || num_time_steps < 1 || num_omegas < 0 || !(rescale > 0.0) || !(kT > 0.0) ||
        !(area_per_orbital > 0.0))
        return TBPM_ERR_ARG;
    const double pi = 3.141592653589793238462643383279;
    const int nt = num_time_steps;
    const double dt = pi / rescale;
    // 2 Im corr(t_k) W(t_k) dt once, then one sine per (w, t)
    std::vector<double> g((size_t)nt + 1);
    for (int k = 0; k <= nt; ++k)
        g[(size_t)k] = 0.5 * (1.0 + std::cos(pi * k / nt)) * 2.0 * corr[2 * k + 1] * dt;
    for (int j = 0; j < num_omegas; ++j) {
        const double w = omegas[j];
        if (!(w > 0.0))
            return TBPM_ERR_ARG;
        double acc = 0.0;
        for (int k = 1; k <= nt; ++k)
            acc += std::sin(w * k * dt) * g[(size_t)k];
        sigma[j] = std::expm1(-w / kT) / (w * area_per_orbital) * acc;
    }
    return TBPM_OK;
}

tbpm_status tbpm_dyn_polarization(const double *corr, int32_t num_time_steps, double rescale,
                                  double area_per_orbital, int32_t num_omegas, const double *omegas, double *pol)
{
    if (!corr || !omegas || !pol || num_time_steps < 1 || num_omegas < 0 || !(rescale > 0.0) ||
        !(area_per_orbital > 0.0))
        return TBPM_ERR_ARG;
    const double pi = 3.141592653589793238462643383279;
    const int nt = num_time_steps;
    const double dt = pi / rescale;
    std::vector<double> g((size_t)nt + 1);
    for (int k = 0; k <= nt; ++k)
        g[(size_t)k] = 0.5 * (1.0 + std::cos(pi * k / nt)) * corr[2 * k + 1] * dt;
    for (int j = 0; j < num_omegas; ++j) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k <= nt; ++k) {
            const double ph = omegas[j] * k * dt;
            re += std::cos(ph) * g[(size_t)k];
            im += std::sin(ph) * g[(size_t)k];
        }
        pol[2 * j] = -2.0 / area_per_orbital * re;
        pol[2 * j + 1] = -2.0 / area_per_orbital * im;
    }
    return TBPM_OK;
}

}  // extern "C"

extern "C" tbpm_status tbpm_patch_plan(const tbpm_csr *csr, int32_t patch_rows, int32_t *new_of_old,
                                       int64_t *num_patches, int32_t *max_halo, double *halo_fraction)
{
    if (!csr || csr->on_device || csr->n < 1 || csr->n > INT32_MAX || !csr->row_ptr || patch_rows < 1 ||
        (csr->nnz > 0 && !csr->col))
        return TBPM_ERR_ARG;
    tbpm::PatchPlan plan;
    tbpm::plan_patches(csr->n, csr->row_ptr, csr->col, patch_rows, INT32_MAX, plan);
    if (new_of_old)
        std::copy(plan.new_of_old.begin(), plan.new_of_old.end(), new_of_old);
    if (num_patches)
        *num_patches = (int64_t)plan.patch_ptr.size() - 1;
    if (max_halo)
        *max_halo = plan.max_halo;
    if (halo_fraction)
        *halo_fraction = plan.halo_fraction;
    return TBPM_OK;
}

extern "C" tbpm_status tbpm_value_table_plan(const tbpm_csr *csr, int32_t dtype, int32_t *entries,
                                            int32_t *per_row_diagonal)
{
    if (!csr || csr->on_device || csr->n < 1 || !csr->row_ptr || (dtype != TBPM_C128 && dtype != TBPM_C64) ||
        (csr->nnz > 0 && (!csr->col || !csr->val)))
        return TBPM_ERR_ARG;
    tbpm::ValueTable vt;
    const bool ok = tbpm::plan_value_table(csr->n, csr->row_ptr, csr->col, csr->val, dtype, vt);
    if (entries)
        *entries = ok ? (int32_t)(vt.keys.size() / 2) : 0;
    if (per_row_diagonal)
        *per_row_diagonal = ok && vt.diag ? (vt.diag_real ? 2 : 1) : 0;
    return TBPM_OK;
}

// ---- host post-processing of moments ------------------------------------------------------

extern "C" {

tbpm_status tbpm_moments_needed(int32_t num_time_steps, double eps, int32_t *num_moments)
{
    if (!num_moments || num_time_steps < 0 || !(eps > 0.0) || !(eps < 1.0))
        return TBPM_ERR_ARG;
    if (num_time_steps == 0) {
        *num_moments = 1;
        return TBPM_OK;
    }
    // the same truncation as one time step's series, at the last time: the
    // first m past x = N_t pi with |J_m(x)| < eps
    const double x = 3.141592653589793238462643383279 * num_time_steps;
    int mmax = (int)std::ceil(x) + 64 + (int)(8.0 * std::cbrt(x));
    std::vector<double> j;
    for (int attempt = 0; attempt < 6; ++attempt, mmax *= 2) {
        if (!bessel_all(x, mmax, j))
            return TBPM_ERR_ARG;
        for (int m = (int)std::floor(x) + 1; m <= mmax; ++m)
            if (std::fabs(j[(size_t)m]) < eps) {
                *num_moments = m;
                return TBPM_OK;
            }
    }
    return TBPM_ERR_ARG;
}

tbpm_status tbpm_corr_from_moments(const double *mu, int32_t num_moments, int32_t num_time_steps, double *corr)
{
    if (!mu || !corr || num_moments < 1 || num_time_steps < 0)
        return TBPM_ERR_ARG;
    const double pi = 3.141592653589793238462643383279;
    corr[0] = mu[0];          // J_m(0) = delta_m0
    corr[1] = mu[1];
    std::vector<double> j;
    for (int k = 1; k <= num_time_steps; ++k) {
        if (!bessel_all(pi * k, num_moments - 1, j))
            return TBPM_ERR_ARG;
        // sum over m grouped by m mod 4, where (-i)^m = 1, -i, -1, i
        double re = j[0] * mu[0], im = j[0] * mu[1];
        for (int m = 1; m < num_moments; ++m) {
            const double a = 2.0 * j[(size_t)m];
            const double mr = mu[2 * m], mi = mu[2 * m + 1];
            switch (m & 3) {
            case 0: re += a * mr; im += a * mi; break;
            case 1: re += a * mi; im -= a * mr; break;
            case 2: re -= a * mr; im -= a * mi; break;
            default: re -= a * mi; im += a * mr; break;
            }
        }
        corr[2 * k] = re;
        corr[2 * k + 1] = im;
    }
    return TBPM_OK;
}

tbpm_status tbpm_kpm_dos(const double *mu, int32_t num_moments, double rescale, int32_t num_energies,
                         double *energies, double *dos)
{
    if (!mu || !energies || !dos || num_moments < 1 || num_energies < 1 || !(rescale > 0.0))
        return TBPM_ERR_ARG;
    const double pi = 3.141592653589793238462643383279;
    const int N = num_moments;
    // Jackson damping factors (Weisse et al., Rev. Mod. Phys. 78, 275, eq. 71)
    const double q = pi / (N + 1);
    const double cot_q = std::cos(q) / std::sin(q);
    std::vector<double> gm((size_t)N);
    for (int m = 0; m < N; ++m)
        gm[(size_t)m] = ((N - m + 1) * std::cos(q * m) + std::sin(q * m) * cot_q) / (N + 1);
    // energies at the Chebyshev nodes x_j = cos(theta_j), ascending; T_m(x_j) = cos(m theta_j)
    for (int jj = 0; jj < num_energies; ++jj) {
        const double th = pi * (num_energies - jj - 0.5) / num_energies;
        const double x = std::cos(th);
        // cos(m th) by the rotation recurrence of (cos, sin)
        const double c1 = std::cos(th), s1 = std::sin(th);
        double cm = 1.0, sm = 0.0, acc = gm[0] * mu[0];
        for (int m = 1; m < N; ++m) {
            if ((m & 63) == 0) {               // re-anchor against drift
                cm = std::cos(m * th);
                sm = std::sin(m * th);
            } else {
                const double cn = cm * c1 - sm * s1;
                sm = sm * c1 + cm * s1;
                cm = cn;
            }
            acc += 2.0 * gm[(size_t)m] * mu[2 * m] * cm;
        }
        energies[jj] = rescale * x;
        dos[jj] = acc / (pi * rescale * std::sqrt(1.0 - x * x));
    }
    return TBPM_OK;
}

}  // extern "C"
