/* A plain C consumer of libtbpm: no Python and no PyTorch in the process.
 *
 * Reads a Hamiltonian in CSR form from a binary file
 *   int64 n, int64 nnz, int64 row_ptr[n+1], int32 col[nnz], float64 val[2*nnz]
 * stores it on device 0, and writes to the output file (float64, in order)
 *   corr  complex [R][N_t+1]   random-phase correlation C_r(t_k)
 *   norms         [R][N_t+1]   <psi_r(t_k)|psi_r(t_k)>
 *   dos           [2 N_t]      Hann-windowed DOS of the library's sample average C(t)
 *   mu    complex [R][M]       Chebyshev moments of the same vectors
 *   srv   complex [R][N_t+1]   the same propagation through the request server
 *   mean  complex [N_t+1]      the library's sample average (1/R) sum_r C_r(t_k)
 * then exercises the documented error statuses on malformed input.  Prints
 * one line per check and exits non-zero on the first unexpected status.
 *
 * usage: tbpm_c_client IN OUT RESCALE STEPS VECTORS BLOCK SEED DTYPE FORMAT MOMENTS [SERIES]
 * SERIES: 0 forward recurrence (default), 1 Clenshaw's backward recurrence.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tbpm.h"

#define CHECK(call)                                                                   \
    do {                                                                              \
        tbpm_status s_ = (call);                                                      \
        if (s_ != TBPM_OK) {                                                          \
            fprintf(stderr, "%s failed: %s (%s)\n", #call, tbpm_status_string(s_),     \
                    ctx ? tbpm_last_error(ctx) : "");                                  \
            return 2;                                                                 \
        }                                                                             \
    } while (0)

static void *read_all(FILE *f, size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (p && bytes && fread(p, 1, bytes, f) != bytes) {
        free(p);
        return NULL;
    }
    return p;
}

static int expect(const char *what, tbpm_status got, tbpm_status want) {
    printf("%-40s %s\n", what, got == want ? "ok" : "UNEXPECTED");
    if (got != want) fprintf(stderr, "%s: got %s, want %s\n", what, tbpm_status_string(got), tbpm_status_string(want));
    return got == want ? 0 : 3;
}

int main(int argc, char **argv) {
    if (argc != 11 && argc != 12) {
        fprintf(stderr, "usage: %s IN OUT RESCALE STEPS VECTORS BLOCK SEED DTYPE FORMAT MOMENTS [SERIES]\n", argv[0]);
        return 1;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) { perror(argv[1]); return 1; }
    int64_t hdr[2];
    if (fread(hdr, sizeof hdr, 1, f) != 1) { fprintf(stderr, "short header\n"); return 1; }
    const int64_t n = hdr[0], nnz = hdr[1];
    int64_t *row_ptr = read_all(f, (size_t)(n + 1) * sizeof(int64_t));
    int32_t *col = read_all(f, (size_t)nnz * sizeof(int32_t));
    double *val = read_all(f, (size_t)nnz * 2 * sizeof(double));
    fclose(f);
    if (!row_ptr || !col || !val) { fprintf(stderr, "short CSR file\n"); return 1; }

    tbpm_params p;
    memset(&p, 0, sizeof p);
    p.rescale = atof(argv[3]);
    p.num_time_steps = atoi(argv[4]);
    p.num_vectors = atoi(argv[5]);
    p.block = atoi(argv[6]);
    p.seed = strtoull(argv[7], NULL, 10);
    const int dtype = atoi(argv[8]), format = atoi(argv[9]), num_moments = atoi(argv[10]);
    const int R = p.num_vectors, T1 = p.num_time_steps + 1;
    if (R < 1 || p.num_time_steps < 1 || num_moments < 1) { fprintf(stderr, "bad sizes\n"); return 1; }

    tbpm_ctx *ctx = NULL;
    CHECK(tbpm_ctx_create(0, NULL, NULL, &ctx));
    if (argc == 12)
        CHECK(tbpm_ctx_set_series(ctx, atoi(argv[11])));
    tbpm_csr csr = {n, nnz, row_ptr, col, val, 0};
    tbpm_ham *ham = NULL;
    CHECK(tbpm_build_csr(ctx, &csr, dtype, format, TBPM_BUILD_CHECK_HERMITIAN, &ham));
    int64_t n_out = 0, nnz_out = 0;
    double gersh = 0.0;
    int32_t fmt_out = -1;
    CHECK(tbpm_ham_info(ham, &n_out, &nnz_out, &gersh, NULL, NULL, &fmt_out));
    printf("stored n=%lld nnz=%lld format=%d gershgorin=%.6f\n", (long long)n_out, (long long)nnz_out, fmt_out,
           gersh);

    double *corr = calloc((size_t)R * T1 * 2, sizeof(double));
    double *norms = calloc((size_t)R * T1, sizeof(double));
    double *avg = calloc((size_t)T1 * 2, sizeof(double));
    double *energies = calloc((size_t)2 * p.num_time_steps, sizeof(double));
    double *dos = calloc((size_t)2 * p.num_time_steps, sizeof(double));
    double *mu = calloc((size_t)R * num_moments * 2, sizeof(double));
    double *srv_corr = calloc((size_t)R * T1 * 2, sizeof(double));
    double *srv_avg = calloc((size_t)T1 * 2, sizeof(double));
    double *avg_only = calloc((size_t)T1 * 2, sizeof(double));
    if (!corr || !norms || !avg || !energies || !dos || !mu || !srv_corr || !srv_avg || !avg_only) {
        fprintf(stderr, "oom\n");
        return 1;
    }

    CHECK(tbpm_propagate_dos(ctx, ham, &p, corr, norms, NULL, avg));
    CHECK(tbpm_dos(avg, p.num_time_steps, p.rescale, 1, energies, dos));
    /* the sample average alone, without the per-vector rows */
    CHECK(tbpm_propagate_dos(ctx, ham, &p, NULL, NULL, NULL, avg_only));
    if (memcmp(avg_only, avg, (size_t)T1 * 2 * sizeof(double)) != 0) {
        fprintf(stderr, "sample average differs without the per-vector rows\n");
        return 4;
    }
    CHECK(tbpm_chebyshev_moments(ctx, ham, &p, num_moments, mu));
    printf("propagate, dos, moments                  ok\n");

    /* the same request through the server: results must not depend on the path */
    tbpm_server *srv = NULL;
    CHECK(tbpm_server_create(ctx, (size_t)1 << 34, 4, &srv));
    uint64_t ticket = 0;
    CHECK(tbpm_submit(srv, ham, &p, &ticket));
    tbpm_status st;
    while ((st = tbpm_poll(srv, ticket, srv_corr, (int64_t)R * T1, srv_avg, T1, NULL)) == TBPM_PENDING) {
    }
    CHECK(st);
    int bad = 0;
    bad |= expect("poll with too small a buffer", tbpm_poll(srv, ticket, srv_corr, (int64_t)R * T1 - 1, NULL, 0, NULL),
                  TBPM_ERR_ARG);
    CHECK(tbpm_server_destroy(srv));
    int same = memcmp(srv_corr, corr, (size_t)R * T1 * 2 * sizeof(double)) == 0 &&
               memcmp(srv_avg, avg, (size_t)T1 * 2 * sizeof(double)) == 0;
    printf("%-40s %s\n", "server result equals direct call", same ? "ok" : "DIFFERENT");
    if (!same) return 4;

    FILE *o = fopen(argv[2], "wb");
    if (!o) { perror(argv[2]); return 1; }
    fwrite(corr, sizeof(double), (size_t)R * T1 * 2, o);
    fwrite(norms, sizeof(double), (size_t)R * T1, o);
    fwrite(dos, sizeof(double), (size_t)2 * p.num_time_steps, o);
    fwrite(mu, sizeof(double), (size_t)R * num_moments * 2, o);
    fwrite(srv_corr, sizeof(double), (size_t)R * T1 * 2, o);
    fwrite(avg, sizeof(double), (size_t)T1 * 2, o);
    fclose(o);

    /* documented error statuses */
    tbpm_params q = p;
    q.rescale = 0.5 * gersh;
    bad |= expect("rescale below Gershgorin bound", tbpm_propagate_dos(ctx, ham, &q, corr, NULL, NULL, NULL),
                  TBPM_ERR_RESCALE);
    q = p;
    q.num_vectors = 0;
    bad |= expect("zero vectors", tbpm_propagate_dos(ctx, ham, &q, corr, NULL, NULL, NULL), TBPM_ERR_ARG);
    bad |= expect("null output", tbpm_propagate_dos(ctx, ham, &p, NULL, NULL, NULL, NULL), TBPM_ERR_ARG);
    if (n >= 2 && nnz >= 1) {
        int32_t saved = col[0];
        col[0] = (int32_t)n;                                      /* column out of range */
        tbpm_ham *h2 = NULL;
        bad |= expect("column out of range", tbpm_build_csr(ctx, &csr, dtype, format, 0, &h2), TBPM_ERR_CSR);
        col[0] = saved;
        int64_t r1 = row_ptr[1];
        row_ptr[1] = row_ptr[n] + 1;                              /* row_ptr not monotone */
        bad |= expect("row_ptr not monotone", tbpm_build_csr(ctx, &csr, dtype, format, 0, &h2), TBPM_ERR_CSR);
        row_ptr[1] = r1;
    }

    CHECK(tbpm_ham_destroy(ham));
    CHECK(tbpm_ctx_destroy(ctx));
    free(row_ptr); free(col); free(val);
    free(corr); free(norms); free(avg); free(energies); free(dos); free(mu); free(srv_corr); free(srv_avg);
    free(avg_only);
    printf("done\n");
    return bad;
}
