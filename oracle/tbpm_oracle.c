/*
 * Reference (oracle) implementation of the TBPM density-of-states path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load.  The GPU library never links, includes or calls it, and it
 * shares no code with the GPU library.
 *
 * Everything is plain FP64 on the CPU, one vector at a time, written to be
 * checked by eye against the method (TBPLaS 2.0, section "Migration to C++"):
 *
 *   e^{-i H dt} psi = sum_{m<M} c_m T_m(H/rho) psi,
 *   c_0 = J_0(tau),  c_m = 2 (-i)^m J_m(tau),  tau = rho * dt,
 *
 * evaluated with the Chebyshev three-term recurrence
 *   p_0 = psi,  p_1 = (H/rho) psi,  p_m = 2 (H/rho) p_{m-1} - p_{m-2},
 * where each new p_m is formed in place of p_{m-2} ("amxsy": y <- a M x - y
 * with a = 2) and then added to the output with its coefficient ("axpy"),
 * the imaginary factor of the time step being folded into c_m.
 *
 * Readings taken where the paper is silent:
 *   dt = pi / rho (so tau = pi), M = first m > tau with |J_m(tau)| < eps,
 *   C(t_k) = <psi0 | psi(t_k)>, k = 0..N_t, random phases from SplitMix64,
 *   DOS = Hann-windowed cosine transform of C on 2 N_t energies in [-rho, rho).
 *
 * Bessel values come from the C library's jn(); the GPU library computes its
 * own with a different method.
 */
#define _DEFAULT_SOURCE
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014; reference splitmix64.c).    */
/* The generator advances its state by the golden-ratio increment and        */
/* returns a bijective 64-bit mix of the new state.                          */
/* ------------------------------------------------------------------------ */
static const uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ull;

static uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Next output of a SplitMix64 generator whose state is *state. */
uint64_t oracle_splitmix64_next(uint64_t *state)
{
    *state += SM_GAMMA;
    return sm_mix(*state);
}

/*
 * Uniform number in [0, 1) for element i of random vector r.
 * The vector's key is output r+1 of SplitMix64 seeded with `seed`; the
 * element's draw is output i+1 of SplitMix64 seeded with that key, whose top
 * 53 bits are scaled by 2^-53.
 */
double oracle_phase_u(uint64_t seed, int64_t r, int64_t i)
{
    uint64_t s = seed;
    uint64_t key = 0;
    for (int64_t k = 0; k <= r; ++k)
        key = oracle_splitmix64_next(&s);
    uint64_t e = key;
    uint64_t out = 0;
    for (int64_t k = 0; k <= i; ++k)
        out = oracle_splitmix64_next(&e);
    return (double)(out >> 11) * 0x1.0p-53;
}

/*
 * Random-phase initial state: psi0[i] = exp(2 pi i u_i) / sqrt(n).
 * (Random samples of TBPM: `num_random_samples`, section "Usage of TBPM solver".)
 * Computed element by element in closed form (the key is found once).
 */
void oracle_random_state(int64_t n, uint64_t seed, int64_t r, double *psi0_out)
{
    cplx *psi0 = (cplx *)psi0_out;
    uint64_t s = seed;
    uint64_t key = 0;
    for (int64_t k = 0; k <= r; ++k)
        key = oracle_splitmix64_next(&s);
    const double amp = 1.0 / sqrt((double)n);
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t i = 0; i < n; ++i) {
        /* output i+1 of the element stream: mix(key + (i+1) * gamma) */
        uint64_t bits = sm_mix(key + (uint64_t)(i + 1) * SM_GAMMA);
        double u = (double)(bits >> 11) * 0x1.0p-53;
        double th = two_pi * u;
        psi0[i] = amp * (cos(th) + I * sin(th));
    }
}

/* ------------------------------------------------------------------------ */
/* Chebyshev coefficients of exp(-i tau x) (Jacobi-Anger expansion).         */
/* ------------------------------------------------------------------------ */

/*
 * Writes c_m, m = 0..M-1, as interleaved complex into coeff[2*max_terms] and
 * returns M, the first m > tau with |J_m(tau)| < eps (so the last kept term
 * is the first one at or above eps past the turning point).  Returns -1 if
 * max_terms is too small.
 */
int oracle_coefficients(double tau, double eps, int max_terms, double *coeff_out)
{
    cplx *coeff = (cplx *)coeff_out;
    int M = -1;
    for (int m = 0; m < max_terms + 1; ++m) {
        double j = jn(m, tau);
        if ((double)m > tau && fabs(j) < eps) {
            M = m;
            break;
        }
        if (m == max_terms)
            break;
        /* (-i)^m cycles 1, -i, -1, i */
        cplx phase;
        switch (m & 3) {
        case 0: phase = 1.0; break;
        case 1: phase = -I; break;
        case 2: phase = -1.0; break;
        default: phase = I; break;
        }
        coeff[m] = (m == 0 ? 1.0 : 2.0) * phase * j;
    }
    return M;
}

/* ------------------------------------------------------------------------ */
/* Validation: Hermiticity and the Gershgorin bound of the spectrum.         */
/* ------------------------------------------------------------------------ */

/* max_i sum_j |H_ij|: every eigenvalue lies in [-g, g]. */
double oracle_gershgorin(int64_t n, const int64_t *row_ptr, const double *val_in)
{
    const cplx *val = (const cplx *)val_in;
    double g = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            s += cabs(val[k]);
        if (s > g)
            g = s;
    }
    return g;
}

/* Entry H_ij (0 if absent), by linear search in row i. */
static cplx csr_entry(const int64_t *row_ptr, const int32_t *col, const cplx *val, int64_t i, int64_t j)
{
    cplx s = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
        if (col[k] == j)
            s += val[k];
    return s;
}

/* 1 if every H_ij equals conj(H_ji) within tol * max|H|, else 0. */
int oracle_is_hermitian(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_in, double tol)
{
    const cplx *val = (const cplx *)val_in;
    double hmax = 0.0;
    for (int64_t k = 0; k < row_ptr[n]; ++k)
        if (cabs(val[k]) > hmax)
            hmax = cabs(val[k]);
    int ok = 1;
#pragma omp parallel for schedule(static) reduction(&& : ok)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int64_t j = col[k];
            if (j < 0 || j >= n) { ok = 0; continue; }
            cplx hij = csr_entry(row_ptr, col, val, i, j);
            cplx hji = csr_entry(row_ptr, col, val, j, i);
            if (cabs(hij - conj(hji)) > tol * hmax)
                ok = 0;
        }
    }
    return ok;
}

/* ------------------------------------------------------------------------ */
/* Sparse and vector kernels, plain loops.                                   */
/* ------------------------------------------------------------------------ */

/* y = s * (H x) */
static void spmv(int64_t n, const int64_t *row_ptr, const int32_t *col, const cplx *val, double s,
                 const cplx *x, cplx *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        cplx acc = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            acc += val[k] * x[col[k]];
        y[i] = s * acc;
    }
}

/* y = s * (H x) - y   (the paper's amxsy, with the 1/rho of H/rho folded into s) */
static void amxsy(int64_t n, const int64_t *row_ptr, const int32_t *col, const cplx *val, double s,
                  const cplx *x, cplx *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        cplx acc = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            acc += val[k] * x[col[k]];
        y[i] = s * acc - y[i];
    }
}

/* y = y + a x */
static void axpy(int64_t n, cplx a, const cplx *x, cplx *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        y[i] += a * x[i];
}

/* <a|b> = sum conj(a_i) b_i, sequential */
static cplx dotc(int64_t n, const cplx *a, const cplx *b)
{
    cplx s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += conj(a[i]) * b[i];
    return s;
}

static double norm2(int64_t n, const cplx *a)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Propagation and correlation function.                                     */
/* ------------------------------------------------------------------------ */

/*
 * Propagates psi0 under H for num_steps steps of length dt and records
 *   corr[k]  = <psi0 | psi(t_k)>          (complex, k = 0..num_steps)
 *   norms[k] = <psi(t_k) | psi(t_k)>      (optional)
 *   site_corr[s][k] = conj(psi0[site_s]) * psi(t_k)[site_s]   (optional)
 * psi_final (optional) receives psi(t_{num_steps}).
 *
 * Returns M (number of Chebyshev coefficients) or a negative error:
 *   -1 bad argument, -2 rescale below the Gershgorin bound, -3 no memory,
 *   -4 coefficient table too small.
 */
/* One time step: psi <- sum_{m<M} c_m T_m(H/rho) psi, with scratch p0, p1. */
static void time_step(int64_t n, const int64_t *row_ptr, const int32_t *col, const cplx *val, const cplx *c,
                      int M, double inv_rho, double two_inv_rho, cplx *psi, cplx *p0, cplx *p1)
{
    memcpy(p0, psi, sizeof(cplx) * (size_t)n);                 /* p0 = T_0 psi          */
    spmv(n, row_ptr, col, val, inv_rho, p0, p1);               /* p1 = T_1 psi          */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        psi[i] = c[0] * p0[i] + c[1] * p1[i];                  /* out = c0 p0 + c1 p1   */
    for (int m = 2; m < M; ++m) {
        /* p0 <- 2 (H/rho) p1 - p0 makes p0 = T_m psi; then out += c_m T_m psi */
        amxsy(n, row_ptr, col, val, two_inv_rho, p1, p0);
        axpy(n, c[m], p0, psi);
        cplx *t = p0; p0 = p1; p1 = t;                          /* rotate roles          */
    }
}

int oracle_propagate(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_in,
                     double rescale, double dt, double eps, int num_steps, const double *psi0_in,
                     double *corr_out, double *norms, int64_t num_sites, const int64_t *sites,
                     double *site_corr_out, double *psi_final_out)
{
    enum { MAX_TERMS = 4096 };
    const cplx *val = (const cplx *)val_in;
    const cplx *psi0 = (const cplx *)psi0_in;
    cplx *corr = (cplx *)corr_out;
    cplx *site_corr = (cplx *)site_corr_out;
    if (n <= 0 || num_steps < 0 || !(rescale > 0.0) || !(dt > 0.0) || !(eps > 0.0))
        return -1;
    if (rescale < oracle_gershgorin(n, row_ptr, val_in))
        return -2;

    double *cbuf = (double *)malloc(sizeof(double) * 2 * MAX_TERMS);
    cplx *psi = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *p0 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *p1 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!cbuf || !psi || !p0 || !p1) {
        free(cbuf); free(psi); free(p0); free(p1);
        return -3;
    }
    const double tau = rescale * dt;
    const int M = oracle_coefficients(tau, eps, MAX_TERMS, cbuf);
    if (M < 2) {
        free(cbuf); free(psi); free(p0); free(p1);
        return -4;
    }
    const cplx *c = (const cplx *)cbuf;
    const double inv_rho = 1.0 / rescale;
    const double two_inv_rho = 2.0 / rescale;

    memcpy(psi, psi0, sizeof(cplx) * (size_t)n);
    for (int k = 0;; ++k) {
        corr[k] = dotc(n, psi0, psi);
        if (norms)
            norms[k] = norm2(n, psi);
        for (int64_t s = 0; s < num_sites; ++s) {
            int64_t i = sites[s];
            site_corr[s * (int64_t)(num_steps + 1) + k] = conj(psi0[i]) * psi[i];
        }
        if (k == num_steps)
            break;
        time_step(n, row_ptr, col, val, c, M, inv_rho, two_inv_rho, psi, p0, p1);
    }
    if (psi_final_out)
        memcpy(psi_final_out, psi, sizeof(cplx) * (size_t)n);
    free(cbuf); free(psi); free(p0); free(p1);
    return M;
}

/* ------------------------------------------------------------------------ */
/* Density of states from the correlation function.                          */
/* ------------------------------------------------------------------------ */

/*
 * d(E) = (1/2pi) int e^{iEt} C(t) dt with C(-t) = conj(C(t)), sampled at
 * E_j = -rho + j rho / N_t, j = 0..2N_t-1, on t_k = k dt with dt = pi/rho:
 *   d_j = dt/(2 pi) [ w_0 Re C_0 + 2 sum_{k=1}^{N_t} w_k Re(C_k e^{i E_j t_k}) ],
 * w_k = (1 + cos(pi k / N_t)) / 2 when window = 1, else 1.
 */
int oracle_dos(const double *corr_in, int num_steps, double rescale, int window,
               double *energies, double *dos)
{
    const cplx *corr = (const cplx *)corr_in;
    if (num_steps < 1 || !(rescale > 0.0))
        return -1;
    const double pi = 3.141592653589793238462643383279;
    const double dt = pi / rescale;
    const int nt = num_steps;
    for (int j = 0; j < 2 * nt; ++j) {
        double e = -rescale + (double)j * rescale / (double)nt;
        double acc = creal(corr[0]);      /* w_0 = 1 */
        for (int k = 1; k <= nt; ++k) {
            double w = window ? 0.5 * (1.0 + cos(pi * (double)k / (double)nt)) : 1.0;
            double ph = e * (double)k * dt;
            acc += 2.0 * w * creal(corr[k] * (cos(ph) + I * sin(ph)));
        }
        energies[j] = e;
        dos[j] = dt / (2.0 * pi) * acc;
    }
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from now on (timing runs only; results do
 * not depend on it: the sums over rows are sequential). */
void oracle_set_num_threads(int threads)
{
#ifdef _OPENMP
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
}

/* ------------------------------------------------------------------------ */
/* Chebyshev moments (kernel polynomial method, TBPLaS "KPM" capability).    */
/* ------------------------------------------------------------------------ */

/*
 * mu_m = <psi0 | T_m(H/rho) | psi0>, m = 0..num_moments-1, by the plain
 * recurrence T_0 psi0 = psi0, T_1 psi0 = (H/rho) psi0,
 * T_m psi0 = 2 (H/rho) T_{m-1} psi0 - T_{m-2} psi0, one inner product per m.
 * mu is written as interleaved complex (the imaginary parts vanish for
 * Hermitian H up to rounding).  Returns 0, or -1 / -2 / -3 as propagate.
 */
int oracle_moments(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_in, double rescale,
                   const double *psi0_in, int num_moments, double *mu_out)
{
    const cplx *val = (const cplx *)val_in;
    const cplx *psi0 = (const cplx *)psi0_in;
    cplx *mu = (cplx *)mu_out;
    if (n <= 0 || num_moments < 1 || !(rescale > 0.0))
        return -1;
    if (rescale < oracle_gershgorin(n, row_ptr, val_in))
        return -2;
    cplx *p0 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *p1 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!p0 || !p1) {
        free(p0); free(p1);
        return -3;
    }
    memcpy(p0, psi0, sizeof(cplx) * (size_t)n);
    mu[0] = dotc(n, psi0, p0);
    if (num_moments > 1) {
        spmv(n, row_ptr, col, val, 1.0 / rescale, p0, p1);
        mu[1] = dotc(n, psi0, p1);
    }
    for (int m = 2; m < num_moments; ++m) {
        amxsy(n, row_ptr, col, val, 2.0 / rescale, p1, p0);    /* p0 <- T_m psi0 */
        mu[m] = dotc(n, psi0, p0);
        cplx *t = p0; p0 = p1; p1 = t;
    }
    free(p0); free(p1);
    return 0;
}

/*
 * C(t_k) = <psi0| exp(-i H t_k) |psi0> from the moments, t_k = k pi / rho:
 * exp(-i x y) = sum_m (2 - delta_m0) (-i)^m J_m(x) T_m(y) with x = rho t_k = k pi,
 * summed over the available moments.  Returns 0 or -1.
 */
int oracle_corr_from_moments(const double *mu_in, int num_moments, int num_steps, double *corr_out)
{
    const cplx *mu = (const cplx *)mu_in;
    cplx *corr = (cplx *)corr_out;
    if (num_moments < 1 || num_steps < 0)
        return -1;
    const double pi = 3.141592653589793238462643383279;
    for (int k = 0; k <= num_steps; ++k) {
        const double x = pi * (double)k;
        cplx s = 0.0;
        for (int m = 0; m < num_moments; ++m) {
            const double j = (k == 0) ? (m == 0 ? 1.0 : 0.0) : jn(m, x);
            cplx phase;
            switch (m & 3) {
            case 0: phase = 1.0; break;
            case 1: phase = -I; break;
            case 2: phase = -1.0; break;
            default: phase = I; break;
            }
            s += (m == 0 ? 1.0 : 2.0) * phase * j * mu[m];
        }
        corr[k] = s;
    }
    return 0;
}

/*
 * Kernel-polynomial DOS with the Jackson kernel (Weisse, Wellein, Alvermann &
 * Fehske, Rev. Mod. Phys. 78, 275 (2006), section II.C): with N moments,
 * g_m = [(N - m + 1) cos(pi m / (N + 1)) + sin(pi m / (N + 1)) cot(pi / (N + 1))] / (N + 1),
 * d(E) = [g_0 mu_0 + 2 sum_{m>=1} g_m mu_m T_m(x)] / (pi rho sqrt(1 - x^2)), x = E / rho,
 * at num_energies points E_j = rho cos(pi (j + 1/2) / num_energies) (Chebyshev
 * nodes, ascending order on output).  Returns 0 or -1.
 */
int oracle_kpm_dos(const double *mu_in, int num_moments, double rescale, int num_energies, double *energies,
                   double *dos)
{
    const cplx *mu = (const cplx *)mu_in;
    if (num_moments < 1 || num_energies < 1 || !(rescale > 0.0))
        return -1;
    const double pi = 3.141592653589793238462643383279;
    const double N = (double)num_moments;
    for (int j = 0; j < num_energies; ++j) {
        const int jj = num_energies - 1 - j;               /* ascending energies */
        const double th = pi * ((double)jj + 0.5) / (double)num_energies;
        const double x = cos(th);
        double acc = 0.0;
        for (int m = 0; m < num_moments; ++m) {
            const double a = pi * (double)m / (N + 1.0);
            const double g = ((N - m + 1.0) * cos(a) + sin(a) * cos(pi / (N + 1.0)) / sin(pi / (N + 1.0))) / (N + 1.0);
            acc += (m == 0 ? 1.0 : 2.0) * g * creal(mu[m]) * cos((double)m * th);   /* T_m(cos th) */
        }
        energies[j] = rescale * x;
        dos[j] = acc / (pi * rescale * sqrt(1.0 - x * x));
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Time-dependent wave function and quasi-eigenstates.                       */
/* ------------------------------------------------------------------------ */

/*
 * Propagates psi0 for num_steps steps of dt = pi / rho (the same time steps as
 * oracle_propagate) and returns
 *   snaps [num_snaps][n]: psi(t_k) at k = snap_steps[s] (each in 0..num_steps);
 *   qe [num_energies][n]: q_j = sum_{k=0}^{N_t} w_k exp(i E_j t_k) psi(t_k),
 *       w_k = (1 + cos(pi k / N_t)) / 2 (w_k = 1 for N_t = 0), t_k = k dt.
 * Either output may be NULL.  Returns M, or -1 (arguments), -2 (rescale below
 * the Gershgorin bound), -3 (memory), -4 (series).
 */
int oracle_propagate_outputs(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_in,
                             double rescale, double eps, int num_steps, const double *psi0_in, int num_snaps,
                             const int32_t *snap_steps, double *snaps_out, int num_energies,
                             const double *energies, double *qe_out)
{
    enum { MAX_TERMS = 4096 };
    const cplx *val = (const cplx *)val_in;
    cplx *snaps = (cplx *)snaps_out;
    cplx *qe = (cplx *)qe_out;
    if (n <= 0 || num_steps < 0 || !(rescale > 0.0) || !(eps > 0.0) || num_snaps < 0 || num_energies < 0)
        return -1;
    for (int s = 0; s < num_snaps; ++s)
        if (snap_steps[s] < 0 || snap_steps[s] > num_steps)
            return -1;
    if (rescale < oracle_gershgorin(n, row_ptr, val_in))
        return -2;
    double *cbuf = (double *)malloc(sizeof(double) * 2 * MAX_TERMS);
    cplx *psi = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *p0 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *p1 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!cbuf || !psi || !p0 || !p1) {
        free(cbuf); free(psi); free(p0); free(p1);
        return -3;
    }
    const double pi = 3.141592653589793238462643383279;
    const double dt = pi / rescale;
    const int M = oracle_coefficients(pi, eps, MAX_TERMS, cbuf);
    if (M < 2) {
        free(cbuf); free(psi); free(p0); free(p1);
        return -4;
    }
    if (qe)
        memset(qe, 0, sizeof(cplx) * (size_t)n * (size_t)num_energies);
    memcpy(psi, psi0_in, sizeof(cplx) * (size_t)n);
    for (int k = 0;; ++k) {
        for (int s = 0; s < num_snaps; ++s)
            if (snap_steps[s] == k)
                memcpy(snaps + (size_t)s * n, psi, sizeof(cplx) * (size_t)n);
        if (qe) {
            const double w = num_steps > 0 ? 0.5 * (1.0 + cos(pi * (double)k / (double)num_steps)) : 1.0;
            for (int j = 0; j < num_energies; ++j) {
                const double ph = energies[j] * (double)k * dt;
                axpy(n, w * (cos(ph) + I * sin(ph)), psi, qe + (size_t)j * n);
            }
        }
        if (k == num_steps)
            break;
        time_step(n, row_ptr, col, val, (const cplx *)cbuf, M, 1.0 / rescale, 2.0 / rescale, psi, p0, p1);
    }
    free(cbuf); free(psi); free(p0); free(p1);
    return M;
}

/* ------------------------------------------------------------------------ */
/* Response functions: AC conductivity and dynamic polarization              */
/* (Kubo formula evaluated by propagation, Yuan, Roldan & Katsnelson,        */
/* Phys. Rev. B 82, 115448 (2010) and 84, 035439 (2011)).                    */
/* ------------------------------------------------------------------------ */

/* Fermi-Dirac occupation f(E) = 1 / (1 + exp((E - mu) / kT)), kT > 0. */
static double fermi(double e, double mu, double kT)
{
    const double x = (e - mu) / kT;
    if (x > 0.0)
        return exp(-x) / (1.0 + exp(-x));
    return 1.0 / (1.0 + exp(x));
}

/*
 * Chebyshev coefficients of f(rho x) on [-1, 1] by Chebyshev-Gauss quadrature
 * with K = 8 max_terms nodes theta_k = pi (k + 1/2) / K:
 *   a_m = (2 - delta_m0) / K sum_k f(rho cos theta_k) cos(m theta_k).
 * Writes a_m, m < M, to coeff (real) and returns M = 1 + the last m < max_terms
 * with |a_m| >= eps, or -1 on bad arguments or when the coefficients have not
 * fallen below eps by m = max_terms - 1.
 */
int oracle_fermi_coefficients(double rescale, double mu, double kT, double eps, int max_terms, double *coeff)
{
    if (!(rescale > 0.0) || !(kT > 0.0) || !(eps > 0.0) || max_terms < 2)
        return -1;
    const double pi = 3.141592653589793238462643383279;
    const int K = 8 * max_terms;
    double *fk = (double *)malloc(sizeof(double) * (size_t)K);
    if (!fk)
        return -1;
    for (int k = 0; k < K; ++k)
        fk[k] = fermi(rescale * cos(pi * (k + 0.5) / K), mu, kT);
    int last = -1;
    for (int m = 0; m < max_terms; ++m) {
        double s = 0.0;
        /* m theta_k = pi m (2k + 1) / (2K): the angle is reduced modulo 2 pi in
         * integers before the cosine, so large m keep full accuracy */
        for (int k = 0; k < K; ++k) {
            const long long j = ((long long)m * (2LL * k + 1)) % (4LL * K);
            s += fk[k] * cos(pi * (double)j / (2.0 * K));
        }
        coeff[m] = (m == 0 ? 1.0 : 2.0) * s / K;
        if (fabs(coeff[m]) >= eps)
            last = m;
    }
    free(fk);
    if (last >= max_terms - 1)
        return -1;
    return last + 1 > 1 ? last + 1 : 1;       /* f = 0 to within eps: one (zero) term */
}

/* y = sum_{m<M} a_m T_m(H/rho) x, a real; plain recurrence with scratch p0, p1 */
static void real_series(int64_t n, const int64_t *row_ptr, const int32_t *col, const cplx *val, double rescale,
                        const double *a, int M, const cplx *x, cplx *y, cplx *p0, cplx *p1)
{
    memcpy(p0, x, sizeof(cplx) * (size_t)n);
    spmv(n, row_ptr, col, val, 1.0 / rescale, p0, p1);
    for (int64_t i = 0; i < n; ++i)
        y[i] = a[0] * p0[i] + (M > 1 ? a[1] * p1[i] : 0.0);
    for (int m = 2; m < M; ++m) {
        amxsy(n, row_ptr, col, val, 2.0 / rescale, p1, p0);
        axpy(n, a[m], p0, y);
        cplx *t = p0; p0 = p1; p1 = t;
    }
}

/*
 * corr(t_k) = <phi2(t_k)| A |phi1(t_k)>, k = 0..num_steps, t_k = k pi / rho, with
 *   phi2(t) = exp(-iHt) f(H) phi,   phi1(t) = exp(-iHt) [1 - f(H)] B phi,
 * f(H) by its Chebyshev series (oracle_fermi_coefficients with eps fermi_eps)
 * and each time step by the propagator's series.  A and B are CSR operators.
 * Returns the number of Fermi terms, or -1 (arguments), -2 (rescale), -3
 * (memory), -4 (series).
 */
int oracle_response_corr(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_in,
                         double rescale, double eps, int num_steps, const double *phi_in,
                         const int64_t *a_rp, const int32_t *a_col, const double *a_val_in,
                         const int64_t *b_rp, const int32_t *b_col, const double *b_val_in,
                         double mu, double kT, double fermi_eps, double *corr_out)
{
    enum { MAX_TERMS = 4096, MAX_FERMI = 16384 };
    const cplx *val = (const cplx *)val_in;
    const cplx *phi = (const cplx *)phi_in;
    const cplx *a_val = (const cplx *)a_val_in;
    const cplx *b_val = (const cplx *)b_val_in;
    cplx *corr = (cplx *)corr_out;
    if (n <= 0 || num_steps < 0 || !(rescale > 0.0) || !(eps > 0.0) || !(kT > 0.0))
        return -1;
    if (rescale < oracle_gershgorin(n, row_ptr, val_in))
        return -2;
    double *fa = (double *)malloc(sizeof(double) * MAX_FERMI);
    double *fb = (double *)malloc(sizeof(double) * MAX_FERMI);
    double *cbuf = (double *)malloc(sizeof(double) * 2 * MAX_TERMS);
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *s1 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *s2 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *p0 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *p1 = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    int ret = -3;
    if (!fa || !fb || !cbuf || !w || !s1 || !s2 || !p0 || !p1)
        goto done;
    ret = -4;
    int MF = -1;
    for (int cap = 256; cap <= MAX_FERMI && MF < 0; cap *= 2)
        MF = oracle_fermi_coefficients(rescale, mu, kT, fermi_eps, cap, fa);
    const int M = oracle_coefficients(3.141592653589793238462643383279, eps, MAX_TERMS, cbuf);
    if (MF < 1 || M < 2)
        goto done;
    /* 1 - f: coefficients delta_m0 - a_m */
    for (int m = 0; m < MF; ++m)
        fb[m] = (m == 0 ? 1.0 : 0.0) - fa[m];
    spmv(n, b_rp, b_col, b_val, 1.0, phi, w);                          /* w = B phi           */
    real_series(n, row_ptr, col, val, rescale, fa, MF, phi, s2, p0, p1); /* phi2 = f(H) phi    */
    real_series(n, row_ptr, col, val, rescale, fb, MF, w, s1, p0, p1);   /* phi1 = (1-f) B phi */
    const cplx *c = (const cplx *)cbuf;
    for (int k = 0;; ++k) {
        spmv(n, a_rp, a_col, a_val, 1.0, s1, w);                       /* w = A phi1(t_k)     */
        corr[k] = dotc(n, s2, w);
        if (k == num_steps)
            break;
        time_step(n, row_ptr, col, val, c, M, 1.0 / rescale, 2.0 / rescale, s1, p0, p1);
        time_step(n, row_ptr, col, val, c, M, 1.0 / rescale, 2.0 / rescale, s2, p0, p1);
    }
    ret = MF;
done:
    free(fa); free(fb); free(cbuf); free(w); free(s1); free(s2); free(p0); free(p1);
    return ret;
}

/*
 * Real part of the AC conductivity from the correlation (Yuan et al. 2010):
 *   sigma(w) = (exp(-w / kT) - 1) / (w Omega) int_0^T W(t) sin(w t) 2 Im corr(t) dt,
 * the integral taken as the sum over t_k = k dt, dt = pi / rho, k = 0..N_t, with
 * the Hann window W(t_k) = (1 + cos(pi k / N_t)) / 2 in place of the damping
 * factor; Omega is the area (or volume) per orbital (corr is a per-orbital
 * trace estimate).  Units hbar = e = 1.  Returns 0 or -1.
 */
int oracle_ac_conductivity(const double *corr_in, int num_steps, double rescale, double kT, double omega_area,
                           int num_omegas, const double *omegas, double *sigma)
{
    const cplx *corr = (const cplx *)corr_in;
    if (num_steps < 1 || !(rescale > 0.0) || !(kT > 0.0) || !(omega_area > 0.0))
        return -1;
    const double pi = 3.141592653589793238462643383279;
    const double dt = pi / rescale;
    for (int j = 0; j < num_omegas; ++j) {
        const double w = omegas[j];
        if (!(w > 0.0))
            return -1;
        double acc = 0.0;
        for (int k = 0; k <= num_steps; ++k) {
            const double win = 0.5 * (1.0 + cos(pi * (double)k / (double)num_steps));
            acc += win * sin(w * k * dt) * 2.0 * cimag(corr[k]) * dt;
        }
        sigma[j] = (exp(-w / kT) - 1.0) / (w * omega_area) * acc;
    }
    return 0;
}

/*
 * Dynamic polarization from the density correlation (Yuan et al. 2011):
 *   Pi(q, w) = -(2 / Omega) int_0^T W(t) exp(i w t) Im corr(t) dt,
 * same time grid and window as oracle_ac_conductivity; complex output.
 */
int oracle_dyn_polarization(const double *corr_in, int num_steps, double rescale, double omega_area,
                            int num_omegas, const double *omegas, double *pi_out)
{
    const cplx *corr = (const cplx *)corr_in;
    cplx *out = (cplx *)pi_out;
    if (num_steps < 1 || !(rescale > 0.0) || !(omega_area > 0.0))
        return -1;
    const double pi = 3.141592653589793238462643383279;
    const double dt = pi / rescale;
    for (int j = 0; j < num_omegas; ++j) {
        cplx acc = 0.0;
        for (int k = 0; k <= num_steps; ++k) {
            const double win = 0.5 * (1.0 + cos(pi * (double)k / (double)num_steps));
            const double ph = omegas[j] * k * dt;
            acc += win * (cos(ph) + I * sin(ph)) * cimag(corr[k]) * dt;
        }
        out[j] = -2.0 / omega_area * acc;
    }
    return 0;
}
