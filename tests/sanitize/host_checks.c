/* Host-only functions of the C ABI under AddressSanitizer and
 * UndefinedBehaviorSanitizer: the patch planner on generated lattices, the
 * Chebyshev and Fermi coefficients, the sample average, the DOS, moment and
 * response transforms, and their argument checks.  Built from
 * tbpm_host.cpp, tbpm_bessel.cpp and tbpm_patch.cpp alone (no GPU code).
 * Prints one line per check; exits non-zero on the first failed check (a
 * sanitizer report aborts the run by itself). */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tbpm.h"

#define REQUIRE(cond, what)                                      \
    do {                                                         \
        if (!(cond)) {                                           \
            fprintf(stderr, "check failed: %s\n", what);         \
            return 1;                                            \
        }                                                        \
        printf("%-48s ok\n", what);                              \
    } while (0)

static const double PI = 3.141592653589793;

/* graphene-like L x L cells, two orbitals each: A(a,b) - B(a,b), B(a-1,b),
 * B(a,b-1), periodic; columns sorted within each row */
static int make_lattice(int L, int64_t **rp_out, int32_t **col_out, double **val_out, int64_t *n_out)
{
    const int64_t n = 2LL * L * L;
    int64_t *rp = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *col = malloc(sizeof(int32_t) * (size_t)(3 * n));
    double *val = malloc(sizeof(double) * (size_t)(6 * n));
    if (!rp || !col || !val)
        return 1;
    rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t cell = i / 2, o = i % 2, a = cell / L, b = cell % L;
        int32_t c[3];
        if (o == 0) {
            c[0] = (int32_t)(2 * (a * L + b) + 1);
            c[1] = (int32_t)(2 * (((a + L - 1) % L) * L + b) + 1);
            c[2] = (int32_t)(2 * (a * L + (b + L - 1) % L) + 1);
        } else {
            c[0] = (int32_t)(2 * (a * L + b));
            c[1] = (int32_t)(2 * (((a + 1) % L) * L + b));
            c[2] = (int32_t)(2 * (a * L + (b + 1) % L));
        }
        for (int x = 0; x < 3; ++x)                    /* sort the three columns */
            for (int y = x + 1; y < 3; ++y)
                if (c[y] < c[x]) {
                    int32_t t = c[x];
                    c[x] = c[y];
                    c[y] = t;
                }
        for (int x = 0; x < 3; ++x) {
            col[3 * i + x] = c[x];
            val[2 * (3 * i + x)] = -2.7;
            val[2 * (3 * i + x) + 1] = 0.0;
        }
        rp[i + 1] = 3 * (i + 1);
    }
    *rp_out = rp;
    *col_out = col;
    *val_out = val;
    *n_out = n;
    return 0;
}

int main(void)
{
    /* status strings */
    for (int s = -10; s <= 1; ++s)
        if (!tbpm_status_string(s) || !tbpm_status_string(s)[0])
            return 1;
    printf("%-48s ok\n", "status strings");

    /* patch planner */
    int64_t *rp, n;
    int32_t *col;
    double *val;
    if (make_lattice(48, &rp, &col, &val, &n))
        return 1;
    tbpm_csr csr = {n, 3 * n, rp, col, val, 0};
    int32_t *perm = malloc(sizeof(int32_t) * (size_t)n);
    char *seen = calloc((size_t)n, 1);
    int64_t np = 0;
    int32_t maxh = 0;
    double frac = 0.0;
    for (int pr = 64; pr <= 1024; pr *= 4) {
        REQUIRE(tbpm_patch_plan(&csr, pr, perm, &np, &maxh, &frac) == TBPM_OK, "patch plan");
        memset(seen, 0, (size_t)n);
        int ok = 1;
        for (int64_t i = 0; i < n; ++i) {
            if (perm[i] < 0 || perm[i] >= n || seen[perm[i]])
                ok = 0;
            else
                seen[perm[i]] = 1;
        }
        REQUIRE(ok && np >= (n + pr - 1) / pr && maxh > 0 && frac > 0.0 && frac < 1.0, "plan is a permutation");
    }
    REQUIRE(tbpm_patch_plan(NULL, 64, perm, &np, &maxh, &frac) == TBPM_ERR_ARG, "plan rejects a null CSR");
    REQUIRE(tbpm_patch_plan(&csr, 0, perm, &np, &maxh, &frac) == TBPM_ERR_ARG, "plan rejects zero patch rows");

    /* value table: one hopping (+0 is entry 0); then a distinct value per entry */
    int32_t ent = -1, pdiag = -1;
    REQUIRE(tbpm_value_table_plan(&csr, TBPM_C128, &ent, &pdiag) == TBPM_OK && ent == 2 && pdiag == 0,
            "value table: one hopping");
    REQUIRE(tbpm_value_table_plan(&csr, TBPM_C64, &ent, &pdiag) == TBPM_OK && ent == 2, "value table, complex64");
    for (int64_t j = 0; j < 3 * n; ++j)
        val[2 * j] = -2.7 - 1e-3 * (double)(j % 300);
    REQUIRE(tbpm_value_table_plan(&csr, TBPM_C128, &ent, &pdiag) == TBPM_OK && ent == 0, "value table: too many");
    for (int64_t j = 0; j < 3 * n; ++j)
        val[2 * j] = -2.7;
    REQUIRE(tbpm_value_table_plan(NULL, TBPM_C128, &ent, &pdiag) == TBPM_ERR_ARG, "value table rejects a null CSR");
    REQUIRE(tbpm_value_table_plan(&csr, 5, &ent, &pdiag) == TBPM_ERR_ARG, "value table rejects a bad dtype");

    /* Chebyshev coefficients of exp(-i pi x) */
    double coeff[2 * 64];
    int32_t M = 0;
    REQUIRE(tbpm_coefficients(PI, 1e-14, 64, coeff, &M) == TBPM_OK && M == 20, "coefficients, M = 20");
    REQUIRE(tbpm_coefficients(PI, 1e-14, 5, coeff, &M) == TBPM_ERR_ARG, "coefficients: table too small");
    REQUIRE(tbpm_coefficients(PI, 1e-14, 64, NULL, &M) == TBPM_ERR_ARG, "coefficients: null output");

    /* sample average and DOS of a synthetic correlation */
    const int nt = 64, R = 3;
    double *rows = malloc(sizeof(double) * 2 * R * (nt + 1));
    double mean[2 * 65], e[128], d[128];
    for (int r = 0; r < R; ++r)
        for (int k = 0; k <= nt; ++k) {
            rows[2 * (r * (nt + 1) + k)] = cos(0.3 * k * (r + 1)) * exp(-0.01 * k);
            rows[2 * (r * (nt + 1) + k) + 1] = -sin(0.3 * k * (r + 1)) * exp(-0.01 * k);
        }
    REQUIRE(tbpm_sample_mean(rows, R, nt + 1, mean) == TBPM_OK && fabs(mean[0] - 1.0) < 1e-15, "sample mean");
    REQUIRE(tbpm_sample_mean(rows, 0, nt + 1, mean) == TBPM_ERR_ARG, "sample mean: no rows");
    REQUIRE(tbpm_dos(mean, nt, 9.0, 1, e, d) == TBPM_OK, "dos");
    double sum = 0.0;
    for (int j = 0; j < 2 * nt; ++j)
        sum += d[j] * 9.0 / nt;
    REQUIRE(fabs(sum - mean[0]) < 1e-12, "dos sum rule");
    REQUIRE(tbpm_dos(mean, 0, 9.0, 1, e, d) == TBPM_ERR_ARG, "dos: no time steps");
    REQUIRE(tbpm_dos(mean, nt, 9.0, 2, e, d) == TBPM_ERR_ARG, "dos: bad window");

    /* moments: C(t) from moments and the Jackson DOS */
    int32_t nm = 0;
    REQUIRE(tbpm_moments_needed(16, 1e-14, &nm) == TBPM_OK && nm > 16 * PI, "moments needed");
    double *mu = calloc((size_t)2 * nm, sizeof(double));
    for (int m = 0; m < nm; ++m)
        mu[2 * m] = cos(m * acos(0.3));                 /* one level at x = 0.3 */
    double corr[2 * 17];
    REQUIRE(tbpm_corr_from_moments(mu, nm, 16, corr) == TBPM_OK, "corr from moments");
    for (int k = 0; k <= 16; ++k)
        if (fabs(corr[2 * k] - cos(0.3 * k * PI)) > 1e-10 || fabs(corr[2 * k + 1] + sin(0.3 * k * PI)) > 1e-10)
            return 1;
    printf("%-48s ok\n", "single level: C(t) = exp(-i x t)");
    double ek[256], dk[256];
    REQUIRE(tbpm_kpm_dos(mu, nm, 9.0, 256, ek, dk) == TBPM_OK, "kpm dos");
    REQUIRE(tbpm_kpm_dos(mu, 0, 9.0, 256, ek, dk) == TBPM_ERR_ARG, "kpm dos: no moments");

    /* Fermi coefficients and response transforms */
    double *fc = malloc(sizeof(double) * 16384);
    int32_t nf = 0;
    REQUIRE(tbpm_fermi_coefficients(9.0, 0.0, 0.0259, 1e-14, 16384, fc, &nf) == TBPM_OK && nf > 100,
            "fermi coefficients");
    REQUIRE(tbpm_fermi_coefficients(9.0, 0.0, -1.0, 1e-14, 16384, fc, &nf) == TBPM_ERR_ARG, "fermi: kT <= 0");
    double om[4] = {0.5, 1.0, 2.0, 3.0}, sig[4], pol[8];
    REQUIRE(tbpm_ac_conductivity(mean, nt, 9.0, 0.0259, 0.05, 4, om, sig) == TBPM_OK, "ac conductivity");
    REQUIRE(tbpm_dyn_polarization(mean, nt, 9.0, 0.05, 4, om, pol) == TBPM_OK, "dynamic polarization");

    free(rp); free(col); free(val); free(perm); free(seen); free(rows); free(mu); free(fc);
    printf("done\n");
    return 0;
}
