/* The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: every
 * exported function on a small disordered lattice and a site list, with a
 * final state, snapshots, quasi-eigenstates and response operators, plus
 * the argument checks.  Prints one line per check; exits non-zero on a failed
 * check (a sanitizer report aborts the run by itself). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* the oracle's exported functions (oracle/tbpm_oracle.c) */
uint64_t oracle_splitmix64_next(uint64_t *state);
double oracle_phase_u(uint64_t seed, int64_t r, int64_t i);
void oracle_random_state(int64_t n, uint64_t seed, int64_t r, double *psi0_out);
int oracle_coefficients(double tau, double eps, int max_terms, double *coeff_out);
double oracle_gershgorin(int64_t n, const int64_t *row_ptr, const double *val_in);
int oracle_is_hermitian(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_in, double tol);
int oracle_propagate(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_in, double rescale,
                     double dt, double eps, int num_steps, const double *psi0_in, double *corr_out, double *norms,
                     int64_t num_sites, const int64_t *sites, double *site_corr_out, double *psi_final_out);
int oracle_dos(const double *corr_in, int num_steps, double rescale, int window, double *energies, double *dos);
int oracle_moments(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_in, double rescale,
                   const double *psi0_in, int num_moments, double *mu_out);
int oracle_corr_from_moments(const double *mu_in, int num_moments, int num_steps, double *corr_out);
int oracle_kpm_dos(const double *mu_in, int num_moments, double rescale, int num_energies, double *energies,
                   double *dos);
int oracle_propagate_outputs(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_in,
                             double rescale, double eps, int num_steps, const double *psi0_in, int num_snaps,
                             const int32_t *snap_steps, double *snaps_out, int num_energies, const double *energies,
                             double *qe_out);
int oracle_fermi_coefficients(double rescale, double mu, double kT, double eps, int max_terms, double *coeff);
int oracle_response_corr(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val_in,
                         double rescale, double eps, int num_steps, const double *phi_in, const int64_t *a_rp,
                         const int32_t *a_col, const double *a_val_in, const int64_t *b_rp, const int32_t *b_col,
                         const double *b_val_in, double mu, double kT, double fermi_eps, double *corr_out);
int oracle_ac_conductivity(const double *corr_in, int num_steps, double rescale, double kT, double omega_area,
                           int num_omegas, const double *omegas, double *sigma);
int oracle_dyn_polarization(const double *corr_in, int num_steps, double rescale, double omega_area, int num_omegas,
                            const double *omegas, double *pi_out);

#define REQUIRE(cond, what)                                      \
    do {                                                         \
        if (!(cond)) {                                           \
            fprintf(stderr, "check failed: %s\n", what);         \
            return 1;                                            \
        }                                                        \
        printf("%-48s ok\n", what);                              \
    } while (0)

int main(void)
{
    /* a ring of n sites with hopping -1 and on-site disorder in [-0.5, 0.5]:
     * columns i-1, i, i+1 sorted (a Hermitian tridiagonal matrix with wrap) */
    const int64_t n = 64;
    int64_t rp[65];
    int32_t col[192];
    double val[384];
    int64_t at = 0;
    rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3] = {(i + n - 1) % n, i, (i + 1) % n};
        for (int x = 0; x < 3; ++x)
            for (int y = x + 1; y < 3; ++y)
                if (c[y] < c[x]) {
                    int64_t t = c[x];
                    c[x] = c[y];
                    c[y] = t;
                }
        for (int x = 0; x < 3; ++x) {
            col[at] = (int32_t)c[x];
            val[2 * at] = c[x] == i ? oracle_phase_u(7, 0, i) - 0.5 : -1.0;
            val[2 * at + 1] = 0.0;
            ++at;
        }
        rp[i + 1] = at;
    }
    REQUIRE(oracle_is_hermitian(n, rp, col, val, 1e-14) == 1, "hermitian");
    const double g = oracle_gershgorin(n, rp, val);
    REQUIRE(g > 2.0 && g <= 2.5, "gershgorin bound");
    uint64_t st = 1234567;
    REQUIRE(oracle_splitmix64_next(&st) != 0, "splitmix64");
    double coeff[2 * 64];
    REQUIRE(oracle_coefficients(3.141592653589793, 1e-14, 64, coeff) == 20, "coefficients");
    REQUIRE(oracle_coefficients(3.141592653589793, 1e-14, 5, coeff) < 0, "coefficients: table too small");

    const int nt = 40;
    double psi0[128], corr[2 * 41], norms[41], site_corr[2 * 2 * 41], fin[128];
    int64_t sites[2] = {0, 63};
    oracle_random_state(n, 3, 0, psi0);
    REQUIRE(oracle_propagate(n, rp, col, val, 3.0, 3.141592653589793 / 3.0, 1e-14, nt, psi0, corr, norms, 2, sites,
                             site_corr, fin) > 0, "propagate");
    REQUIRE(fabs(corr[0] - 1.0) < 1e-14 && fabs(norms[nt] - 1.0) < 1e-12, "C(0) = 1, unitarity");
    REQUIRE(oracle_propagate(n, rp, col, val, 1.0, 3.141592653589793, 1e-14, nt, psi0, corr, norms, 0, NULL, NULL,
                             NULL) == -2, "propagate: rescale below the bound");
    double e[80], d[80];
    REQUIRE(oracle_dos(corr, nt, 3.0, 1, e, d) == 0, "dos");
    double mu[2 * 200];
    REQUIRE(oracle_moments(n, rp, col, val, 3.0, psi0, 200, mu) == 0, "moments");
    double c2[2 * 41];
    REQUIRE(oracle_corr_from_moments(mu, 200, 40, c2) == 0, "corr from moments");
    double ek[100], dk[100];
    REQUIRE(oracle_kpm_dos(mu, 200, 3.0, 100, ek, dk) == 0, "kpm dos");
    int32_t snaps_at[3] = {0, 7, nt};
    double snaps[3 * 128], en[2] = {-1.0, 0.5}, qe[2 * 128];
    REQUIRE(oracle_propagate_outputs(n, rp, col, val, 3.0, 1e-14, nt, psi0, 3, snaps_at, snaps, 2, en, qe) > 0,
            "snapshots and quasi-eigenstates");
    REQUIRE(memcmp(snaps, psi0, sizeof(double) * 128) == 0, "snapshot at step 0 is psi0");
    double *fc = malloc(sizeof(double) * 4096);
    REQUIRE(oracle_fermi_coefficients(3.0, 0.0, 0.1, 1e-14, 4096, fc) > 0, "fermi coefficients");
    /* response with A = B = the on-site part of H (a diagonal operator) */
    int64_t drp[65];
    int32_t dcol[64];
    double dval[128];
    for (int64_t i = 0; i < n; ++i) {
        drp[i] = i;
        dcol[i] = (int32_t)i;
        dval[2 * i] = oracle_phase_u(7, 0, i) - 0.5;
        dval[2 * i + 1] = 0.0;
    }
    drp[n] = n;
    double rc[2 * 21];
    REQUIRE(oracle_response_corr(n, rp, col, val, 3.0, 1e-14, 20, psi0, drp, dcol, dval, drp, dcol, dval, 0.0, 0.1,
                                 1e-14, rc) > 0, "response correlation");
    double om[3] = {0.5, 1.0, 2.0}, sig[3], pol[6];
    REQUIRE(oracle_ac_conductivity(rc, 20, 3.0, 0.1, 1.0, 3, om, sig) == 0, "ac conductivity");
    REQUIRE(oracle_dyn_polarization(rc, 20, 3.0, 1.0, 3, om, pol) == 0, "dynamic polarization");
    free(fc);
    printf("done\n");
    return 0;
}
