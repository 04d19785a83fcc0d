/*
 * tbpm.h -- C ABI of the MI355X (gfx950) TBPM propagation library.
 *
 * The library computes the density-of-states correlation function of the
 * tight-binding propagation method (TBPM) as described in TBPLaS 2.0
 * ("Usage of TBPM solver": build a sparse Hamiltonian, set rescale, number
 * of random samples and number of time steps, call calc_corr_dos to obtain
 * C(t), then turn C(t) into a DOS).  A random-phase state psi0 is evolved
 * with the Chebyshev expansion of exp(-i H dt) ("Migration to C++": the
 * three-term recurrence formed in place as y <- 2 (H/rho) x - y, each term
 * accumulated with its coefficient c_m = (2 - delta_m0) (-i)^m J_m(rho dt)),
 * and C(t_k) = <psi0 | psi(t_k)> is recorded at t_k = k dt, k = 0..N_t.
 * tbpm_ctx_set_series selects instead Clenshaw's backward recurrence for the
 * same truncated series (fewer vector passes per term).
 *
 * Conventions fixed by this library where the paper is silent:
 *   dt = pi / rescale; the series keeps m = 0..M-1 where M is the first
 *   m > rho dt with |J_m(rho dt)| < bessel_eps (M = 20 at the default
 *   1e-14, i.e. 19 applications of H per time step);
 *   psi0_r[i] = exp(2 pi i u) / sqrt(n) with u the top 53 bits (times 2^-53)
 *   of output i+1 of SplitMix64 seeded with output r+1 of SplitMix64 seeded
 *   with `seed`;
 *   DOS on E_j = -rho + j rho / N_t, j = 0..2 N_t - 1.
 *
 * General rules:
 *   - every function returns a tbpm_status; no exception crosses the ABI;
 *   - complex numbers are interleaved (re, im) doubles unless stated;
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *     device memory on the context's device;
 *   - the caller owns every array it passes in and every output buffer;
 *     the library owns the objects it returns until the matching destroy;
 *   - a tbpm_ctx is used by one thread at a time; a tbpm_server is safe to
 *     call from several threads.
 */
#ifndef TBPM_H
#define TBPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tbpm_status;
enum {
    TBPM_OK = 0,
    TBPM_PENDING = 1,            /* tbpm_poll: request queued or running          */
    TBPM_ERR_ARG = -1,           /* invalid argument (null pointer, bad size, ...) */
    TBPM_ERR_CSR = -2,           /* CSR malformed: row_ptr not monotone, column out
                                    of range or unsorted, or not Hermitian          */
    TBPM_ERR_RESCALE = -3,       /* rescale below the Gershgorin bound of H         */
    TBPM_ERR_TOO_LARGE = -4,     /* request footprint exceeds the server's budget   */
    TBPM_ERR_OOM = -5,           /* device allocation failed                        */
    TBPM_ERR_DIVERGED = -6,      /* |<psi|psi> - 1| exceeded norm_tol               */
    TBPM_ERR_HIP = -7,           /* HIP runtime error                               */
    TBPM_ERR_CANCELLED = -8,     /* request cancelled                               */
    TBPM_ERR_UNKNOWN = -9        /* unknown ticket                                  */
};

/* Device memory provider.  alloc returns a device pointer of at least `bytes`
 * bytes (NULL on failure); free releases it.  Both may be called from the
 * server's scheduler thread.  Pass NULL to tbpm_ctx_create to use hipMalloc. */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} tbpm_allocator;

typedef struct tbpm_ctx tbpm_ctx;
typedef struct tbpm_ham tbpm_ham;
typedef struct tbpm_server tbpm_server;

/* Storage precision of the Hamiltonian and the vectors.
 *   TBPM_C128: complex128 everywhere (the plain FP64 method);
 *   TBPM_C64:  complex64 H and vectors, FP32 sparse products, the Chebyshev
 *              update (rescale, recurrence, coefficient) in FP64 registers
 *              rounded once to complex64 on store, correlation sums in FP64. */
enum { TBPM_C128 = 0, TBPM_C64 = 1 };
/* Device format: CSR, slot-major ELLPACK, chosen by the library, or ELLPACK
 * over patch-reordered rows (TBPM_FMT_PATCH: rows renumbered so that compact
 * patches of the sparsity graph are contiguous; two Chebyshev terms then
 * share one pass over H, with the first term's result for a patch and its
 * halo kept in on-chip memory).  Results are returned in the caller's
 * original orbital order for every format.  TBPM_FMT_AUTO picks PATCH for
 * matrices of at least 65536 rows whose rows fit ELL (<= 15% padding) with a
 * row length of 3, 4, 5, 8 or 12 and small enough patch halos; else ELL when
 * padding is <= 15%; else CSR.  PATCH falls back the same way. */
enum { TBPM_FMT_CSR = 0, TBPM_FMT_ELL = 1, TBPM_FMT_AUTO = 2, TBPM_FMT_PATCH = 3 };
/* tbpm_build_csr flags: check Hermiticity; use 2048-row instead of 1024-row
 * patches for TBPM_FMT_PATCH when rows hold at most 5 entries; store every
 * entry's value even when a value table applies (see tbpm_ham_value_table) */
enum { TBPM_BUILD_CHECK_HERMITIAN = 1, TBPM_BUILD_LARGE_PATCHES = 2, TBPM_BUILD_NO_VALUE_TABLE = 4 };

/* A Hamiltonian in CSR form (cf. build_ham_csr, TBPLaS 2.0 "Analytical
 * Hamiltonian").  row_ptr: int64 [n+1], row_ptr[0] = 0, non-decreasing,
 * row_ptr[n] = nnz.  col: int32 [nnz], strictly increasing within a row,
 * in [0, n).  val: complex128 [nnz] interleaved (2*nnz doubles), in eV.
 * on_device = 0: the three arrays are host memory; 1: device memory.
 * Caller-owned; the library copies what it needs before tbpm_build_csr
 * returns. */
typedef struct {
    int64_t n;
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col;
    const double *val;
    int32_t on_device;
} tbpm_csr;

/* Propagation parameters (TBPMSolver.config: rescale, num_random_samples,
 * num_time_steps). */
typedef struct {
    double rescale;           /* rho (eV); must be >= the Gershgorin bound of H   */
    int32_t num_time_steps;   /* N_t >= 0; C has N_t + 1 entries per vector       */
    int32_t num_vectors;      /* R >= 1 random-phase vectors                      */
    int32_t block;            /* vectors per SpMM block: 0 = library choice, else
                                 1..64 (processed as powers of two)              */
    int32_t first_vector;     /* index r of the first vector (vectors r0..r0+R-1) */
    uint64_t seed;            /* random-phase seed                                */
    double bessel_eps;        /* truncation threshold; <= 0 means 1e-14           */
    double norm_tol;          /* > 0: fail with TBPM_ERR_DIVERGED when any
                                 |<psi(t_k)|psi(t_k)> - 1| exceeds it; the device
                                 flags it as it happens, so a synchronous call
                                 stops after the block of vectors that shows it
                                 and a served request at the end of the chunk
                                 of steps that shows it; 0: off                   */
    const int64_t *ldos_sites;  /* host, optional: orbital indices for the
                                   per-site correlation (LDOS estimator)          */
    int32_t num_ldos_sites;
    int32_t lanes_per_row;    /* CSR with one vector per block: lanes sharing a
                                 row, 0 = library choice, else 1, 2, 4, 8 or 16  */
} tbpm_params;

/* ---- context -------------------------------------------------------------- */

/* Creates a context on HIP device `device`.  alloc: device memory provider or
 * NULL (hipMalloc).  hip_stream: a hipStream_t the library launches on, or
 * NULL for the library's own stream.  *out receives the context. */
tbpm_status tbpm_ctx_create(int device, const tbpm_allocator *alloc, void *hip_stream, tbpm_ctx **out);
tbpm_status tbpm_ctx_destroy(tbpm_ctx *ctx);
/* Message of the last error on this context (never NULL). */
const char *tbpm_last_error(const tbpm_ctx *ctx);
const char *tbpm_status_string(tbpm_status s);

/* Kernel timing for benchmarks.  While enabled, every time step of the
 * synchronous propagation calls brackets its first Chebyshev term, its run
 * of middle terms and its last term with HIP events on the context's stream
 * and adds the elapsed times to per-kind totals (kind 0: first term,
 * 1: middle terms, 2: last term with the correlation sums).  Enabling resets
 * the totals.  *launches receives the number of kernel launches timed. */
tbpm_status tbpm_ctx_set_profiling(tbpm_ctx *ctx, int32_t enable);
/* HIP graphs for the time steps of tbpm_propagate_dos / _states / _sites:
 * mode 0 never; 1 (default) when the problem is small enough for launch
 * overhead to matter (n x block <= 2^21); 2 whenever possible.  A run uses a
 * graph only without LDOS sites, snapshots and quasi-eigenstates, and
 * with at least 12 steps: 6 consecutive steps are captured once
 * per block width and replayed; results are identical to the launches one by
 * one.  With kernel timing on, a graph launch is timed as a whole and
 * counted as middle-term time over all its term launches (reductions
 * included).  tbpm_ctx_graph_replays: graph launches on this context so far. */
tbpm_status tbpm_ctx_set_graphs(tbpm_ctx *ctx, int32_t mode);
tbpm_status tbpm_ctx_graph_replays(const tbpm_ctx *ctx, int64_t *replays);
/* How the Chebyshev series of a time step (and the Fermi operator's series
 * in tbpm_response_corr) is evaluated on this context:
 *   TBPM_SERIES_FORWARD (default): the paper's forward three-term recurrence,
 *     p_m = 2 (H/rho) p_m-1 - p_m-2, with c_m p_m accumulated into the result;
 *   TBPM_SERIES_CLENSHAW: Clenshaw's backward recurrence for the same
 *     truncated series, b_m = c_m psi + 2 (H/rho) b_m+1 - b_m+2 and
 *     psi(t + dt) = c_0 psi + (H/rho) b_1 - b_2 (series of at least 5 terms;
 *     6 with fused pairs): no accumulator vector, so a product with H
 *     streams one vector fewer.  Results equal the forward recurrence's up
 *     to rounding.
 * Applies to calls started afterwards, server requests included (read when a
 * request starts).  The Chebyshev moments always use the forward recurrence. */
enum { TBPM_SERIES_FORWARD = 0, TBPM_SERIES_CLENSHAW = 1 };
tbpm_status tbpm_ctx_set_series(tbpm_ctx *ctx, int32_t mode);
tbpm_status tbpm_ctx_kernel_time(const tbpm_ctx *ctx, int32_t kind, double *total_ms, int64_t *launches);

/* ---- Hamiltonian ----------------------------------------------------------- */

/* Validates `csr` (TBPM_ERR_CSR on malformed input; with
 * TBPM_BUILD_CHECK_HERMITIAN also H_ij = conj(H_ji) within 1e-14 max|H|),
 * computes its Gershgorin bound max_i sum_j |H_ij|, and stores it on the
 * device in `dtype` (TBPM_C128 / TBPM_C64) and `format` (TBPM_FMT_*).
 * The stored matrix belongs to the library until tbpm_ham_destroy and must
 * outlive every request that uses it. */
tbpm_status tbpm_build_csr(tbpm_ctx *ctx, const tbpm_csr *csr, int32_t dtype, int32_t format,
                           int32_t flags, tbpm_ham **out);
/* Any output pointer may be NULL.  format: TBPM_FMT_CSR or TBPM_FMT_ELL as
 * stored; bytes: device bytes held by the stored matrix. */
tbpm_status tbpm_ham_info(const tbpm_ham *ham, int64_t *n, int64_t *nnz, double *gershgorin,
                          size_t *bytes, int32_t *dtype, int32_t *format);
/* Value table of a TBPM_FMT_PATCH matrix.  The hoppings of a supercell are
 * copies of its primitive cell's few hoppings, so its off-diagonal entries
 * usually take a handful of distinct values.  When they take at most 254
 * nonzero values (compared bit for bit in the stored precision) and the CSR
 * was given in host memory, tbpm_build_csr also stores a table of the
 * distinct values and one byte per entry indexing it; on-site energies that
 * are too many for the table (Anderson disorder) are kept as one value per
 * row.  The fused-pair and staged complex64 kernels then read 1 byte per
 * entry (+ one value per row) instead of the value itself; results are
 * bitwise the same as without the table (TBPM_BUILD_NO_VALUE_TABLE).
 * entries: values in the table, 0 when none is stored; per_row_diagonal: 0
 * when the table holds the diagonal too, 1 when the diagonal is kept per
 * row, 2 when only its real part is (every on-site value real, as in a
 * Hermitian H, with an imaginary part of +0).  Either output may be NULL. */
tbpm_status tbpm_ham_value_table(const tbpm_ham *ham, int32_t *entries, int32_t *per_row_diagonal);
/* Host-only: the value table tbpm_build_csr would store for the host CSR
 * `csr` in precision `dtype` (same outputs as tbpm_ham_value_table; entries
 * 0 when none applies).  No device work; TBPM_ERR_ARG for a device CSR. */
tbpm_status tbpm_value_table_plan(const tbpm_csr *csr, int32_t dtype, int32_t *entries, int32_t *per_row_diagonal);
/* Whether the forward recurrence (the paper's series, "Migration to C++")
 * applies the middle Chebyshev terms of blocks of `block` vectors of `ham`
 * two to a pass over H: *fused = 1 for one vector on TBPM_FMT_PATCH, and for
 * complex64 blocks of 8 or 16 vectors on TBPM_FMT_PATCH with at most 8
 * entries in a row whose patches have halos of at most 1280 rows; else 0
 * (one term per pass).  Series of fewer
 * than 4 terms, and Clenshaw's recurrence on blocks, take single terms
 * whatever this says.  TBPM_ERR_ARG for a null ham or fused, or block < 1. */
tbpm_status tbpm_ham_fused_pairs(const tbpm_ham *ham, int32_t block, int32_t *fused);
tbpm_status tbpm_ham_destroy(tbpm_ham *ham);

/* Autotuner: times one middle Chebyshev term of `ham` on scratch vectors for
 * every candidate shape -- lanes per row 1, 2, 4, 8, 16 (CSR, one vector) and
 * block widths 1, 2, 4, ... up to max_block (a power of two <= 64) -- and
 * picks the fastest per vector.  The chosen lanes per row is stored in `ham`
 * and used whenever params->lanes_per_row is 0; the chosen block width is
 * stored likewise and used whenever params->block is 0 (capped by the
 * number of vectors).  Outputs (each may be NULL): best_lanes, best_block,
 * and us_per_vector_term, the measured microseconds per vector and term.
 * Allocates scratch vectors for max_block vectors for the duration. */
tbpm_status tbpm_autotune(tbpm_ctx *ctx, tbpm_ham *ham, int32_t max_block, int32_t *best_lanes, int32_t *best_block,
                          double *us_per_vector_term);

/* Host-only: the patch plan tbpm_build_csr would use for TBPM_FMT_PATCH on
 * the host CSR `csr` (patches of at most patch_rows rows grown by
 * breadth-first search).  new_of_old (optional, int32 [n]) receives the new
 * index of every row; num_patches, max_halo (largest halo, in rows) and
 * halo_fraction (total halo rows / n) describe the plan.  No device work. */
tbpm_status tbpm_patch_plan(const tbpm_csr *csr, int32_t patch_rows, int32_t *new_of_old, int64_t *num_patches,
                            int32_t *max_halo, double *halo_fraction);

/* Sets the tuning tbpm_autotune would store (e.g. from a saved result):
 * lanes_per_row 1, 2, 4, 8 or 16; block a power of two 1..64, or 0 to clear. */
tbpm_status tbpm_ham_set_tuning(tbpm_ham *ham, int32_t lanes_per_row, int32_t block);

/* Device bytes a propagation of `ham` with `params` allocates beyond the
 * stored matrix (vectors, partial sums, correlation buffers). */
tbpm_status tbpm_footprint(const tbpm_ham *ham, const tbpm_params *params, size_t *bytes);

/* ---- propagation ------------------------------------------------------------ */

/* Chebyshev coefficients of exp(-i tau x) (host, FP64, Miller's backward
 * recurrence for J_m): writes c_m, m = 0..M-1 as complex into
 * coeff[2*max_terms] and M into *num_terms.  TBPM_ERR_ARG if M > max_terms. */
tbpm_status tbpm_coefficients(double tau, double eps, int32_t max_terms, double *coeff, int32_t *num_terms);

/* calc_corr_dos ("Usage of TBPM solver": the correlation function averaged
 * over the random samples): propagates params->num_vectors random-phase
 * vectors on the context's stream and returns, in host memory,
 *   corr      complex [R][N_t+1]: C_r(t_k) = <psi0_r | psi_r(t_k)>  (optional)
 *   norms     double  [R][N_t+1]: <psi_r(t_k) | psi_r(t_k)>         (optional)
 *   ldos_corr complex [S][N_t+1]: (n / R) sum_r conj(psi0_r[i_s]) psi_r(t_k)[i_s]
 *             at the S = params->num_ldos_sites sites             (optional)
 *   corr_mean complex [N_t+1]: the sample average
 *             C(t_k) = (1/R) sum_{r=0}^{R-1} C_r(t_k), summed in FP64 in the
 *             order r = 0..R-1 (independent of the block width)   (optional)
 * At least one of corr and corr_mean must be non-NULL (TBPM_ERR_ARG).
 * Blocks until the results are on the host.  On TBPM_ERR_DIVERGED the outputs
 * are still written: the vectors of the blocks that ran, zeros for the rest
 * (the run stops after the first block whose norms left norm_tol). */
tbpm_status tbpm_propagate_dos(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params,
                               double *corr, double *norms, double *ldos_corr, double *corr_mean);

/* Same propagation from given initial states instead of random phases:
 * psi0 is host complex128 [R][n] (R = params->num_vectors; seed unused).
 * psi_final (optional, host complex128 [R][n]) receives psi_r(t_{N_t}). */
tbpm_status tbpm_propagate_states(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params,
                                  const double *psi0, double *corr, double *norms, double *psi_final);

/* Propagation of site-localised states e_i, i = sites[s] (original orbital
 * index): corr (host complex [num_sites][N_t+1]) receives the exact local
 * correlation C_i(t_k) = <i|e^{-iH t_k}|i>, whose transform (tbpm_dos) is the
 * LDOS of site i; norms (optional, [num_sites][N_t+1]).  Sites run in blocks
 * of params->block; params->num_vectors, first_vector and seed are ignored. */
tbpm_status tbpm_propagate_sites(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params,
                                 const int64_t *sites, int32_t num_sites, double *corr, double *norms);

/* Time-dependent wave function (the paper's TBPM solver benchmarks "WFT"):
 * propagates one state -- psi0 (host complex128 [n]) or, when psi0 is NULL,
 * the random-phase vector of params->seed and first_vector -- for
 * params->num_time_steps steps of dt = pi / rescale, and copies
 * psi(t_k) for k = steps[s] (each in 0..N_t) to snapshots (host complex128
 * [num_snapshots][n], original row order).  params->num_vectors must be 1.
 * corr (optional, complex [N_t+1]) receives C(t_k) = <psi0|psi(t_k)>. */
tbpm_status tbpm_time_evolution(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params, const double *psi0,
                                int32_t num_snapshots, const int32_t *steps, double *snapshots, double *corr);

/* Quasi-eigenstates (the paper's TBPM solver benchmarks "QE"): the same
 * propagation of one state, accumulating on the device (FP64)
 *   qe[j] = sum_{k=0}^{N_t} w_k exp(i E_j t_k) psi(t_k),  E_j = energies[j],
 * t_k = k pi / rescale, w_k = (1 + cos(pi k / N_t)) / 2 (1 when N_t = 0),
 * written unnormalised to qe (host complex128 [num_energies][n], original row
 * order).  It equals sum_n <n|psi0> |n> F(E_j - E_n), F(w) = sum_k w_k e^{i w t_k}:
 * the eigenstates near E_j, filtered.  params->num_vectors must be 1; corr as
 * in tbpm_time_evolution. */
tbpm_status tbpm_quasi_eigenstates(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params,
                                   const double *psi0, int32_t num_energies, const double *energies, double *qe,
                                   double *corr);

/* Host-only: the sample average mean[k] = (1/R) sum_{r=0}^{R-1} rows[r][k],
 * k < len, of R = num_rows complex rows of len entries each (rows: complex
 * [num_rows][len], mean: complex [len]), summed in FP64 in the order
 * r = 0..R-1 -- the average tbpm_propagate_dos returns as corr_mean, here for
 * per-vector results of the other routes (e.g. Chebyshev moments). */
tbpm_status tbpm_sample_mean(const double *rows, int32_t num_rows, int32_t len, double *mean);

/* Analyzer.calc_dos: host-only.  From corr[N_t+1] (complex) computes
 * dos[j] = dt/(2 pi) [w_0 Re C_0 + 2 sum_{k=1}^{N_t} w_k Re(C_k e^{i E_j t_k})]
 * at energies[j] = -rescale + j rescale / N_t, j < 2 N_t, dt = pi / rescale,
 * with w_k = (1 + cos(pi k / N_t)) / 2 for window = 1 (Hann) or 1 for 0. */
tbpm_status tbpm_dos(const double *corr, int32_t num_time_steps, double rescale, int32_t window,
                     double *energies, double *dos);

/* ---- allocation-free propagation ------------------------------------------------- */

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * random-phase propagation as tbpm_propagate_dos (same kernels and launch
 * shapes, results equal to it), with every device buffer taken from a fixed
 * scratch area of TBPM_NOALLOC_MAX_BYTES bytes that the library holds on each
 * device it runs on until the process ends (its address is set up by
 * tbpm_ctx_create).  The call allocates no device memory (no hipMalloc, no
 * call of the context's allocator), no pinned host memory, and uses no HIP
 * graph; ham must have been built beforehand.
 *   corr      host complex [R][N_t+1] (required), norms host [R][N_t+1]
 *             (optional), corr_mean host complex [N_t+1] (optional): as in
 *             tbpm_propagate_dos; LDOS sites are rejected (TBPM_ERR_ARG).
 * TBPM_ERR_TOO_LARGE when the buffers (about 4, with fused term pairs 6,
 * vectors of n x block complex entries, plus (N_t+1) x block x 24 bytes)
 * exceed the scratch area.  Calls share the device's scratch area and keep
 * its last contents: calls that overlap on one device (two threads, or two
 * contexts with different streams) race and must be serialised by the
 * caller.  Nothing in the area needs to start at zero: every buffer is
 * written before it is read. */
#define TBPM_NOALLOC_MAX_BYTES ((size_t)64 << 20)
tbpm_status tbpm_propagate_dos_noalloc(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params,
                                       double *corr, double *norms, double *corr_mean);

/* ---- Chebyshev moments (kernel polynomial method) ------------------------------ */

/* The expansion behind both the propagator and the DOS (TBPLaS 2.0 lists the
 * kernel polynomial method among its solvers; the propagator of "Migration to
 * C++" is the same Chebyshev series at x = pi): for each of params->num_vectors
 * random-phase vectors (the same vectors tbpm_propagate_dos draws for the same
 * seed and first_vector),
 *   mu[r][m] = <psi0_r | T_m(H / rescale) | psi0_r>,  m < num_moments,
 * written to host memory as complex128 [R][num_moments] (the imaginary parts
 * vanish up to rounding).  Computed with ceil(num_moments / 2) products with H
 * per vector by the doubling identities mu_2m = 2 <p_m|p_m> - mu_0 and
 * mu_2m+1 = 2 <p_m|p_m+1> - mu_1, p_m = T_m(H/rescale) psi0.  Uses rescale,
 * num_vectors, block, first_vector, seed and lanes_per_row of params; the
 * time-step fields are ignored and LDOS sites are rejected (TBPM_ERR_ARG).
 * Blocks until the moments are on the host. */
tbpm_status tbpm_chebyshev_moments(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params,
                                   int32_t num_moments, double *mu);
/* Exact local moments (per-site LDOS, as the paper's TBPM solver benchmarks
 * "LDOS"): the same recurrence from the site-localised states e_i,
 *   mu[s][m] = <i_s | T_m(H / rescale) | i_s>,  i_s = sites[s] (original
 * orbital index, 0 <= i_s < n), host complex128 [num_sites][num_moments];
 * the LDOS of site i_s is tbpm_kpm_dos of row s.  Sites are processed in
 * blocks of params->block (0: the library's choice); params->num_vectors,
 * first_vector and seed are ignored. */
tbpm_status tbpm_site_moments(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params, const int64_t *sites,
                              int32_t num_sites, int32_t num_moments, double *mu);
/* Device bytes tbpm_chebyshev_moments allocates beyond the stored matrix. */
tbpm_status tbpm_moments_footprint(const tbpm_ham *ham, const tbpm_params *params, int32_t num_moments,
                                   size_t *bytes);
/* Host-only: the number of moments whose series reaches C(t) at every
 * t_k = k pi / rescale, k <= num_time_steps, to the truncation eps: the first
 * m > N_t pi with |J_m(N_t pi)| < eps (1 for N_t = 0). */
tbpm_status tbpm_moments_needed(int32_t num_time_steps, double eps, int32_t *num_moments);
/* Host-only: C(t_k) = sum_m (2 - delta_m0) (-i)^m J_m(k pi) mu_m, k = 0..N_t,
 * from one vector's (or an average of) moments mu complex [num_moments];
 * corr: complex [N_t+1], t_k = k pi / rescale as in tbpm_propagate_dos. */
tbpm_status tbpm_corr_from_moments(const double *mu, int32_t num_moments, int32_t num_time_steps, double *corr);
/* Host-only: kernel-polynomial DOS with the Jackson kernel,
 * d(E) = [g_0 mu_0 + 2 sum_{m>=1} g_m Re mu_m T_m(x)] / (pi rescale sqrt(1 - x^2)),
 * x = E / rescale, g_m = [(N-m+1) cos(m q) + sin(m q) cot q] / (N+1),
 * q = pi / (N+1), N = num_moments, at the num_energies Chebyshev nodes
 * E_j = rescale cos(pi (K - j - 1/2) / K), K = num_energies, ascending. */
tbpm_status tbpm_kpm_dos(const double *mu, int32_t num_moments, double rescale, int32_t num_energies,
                         double *energies, double *dos);

/* ---- response functions: AC conductivity, dynamic polarization ----------------- */

/* Stores an operator A (a CSR of the same dimension as ref's H, host memory
 * when ref is patch-reordered) for tbpm_response_corr: as a CSR in ref's
 * dtype and in ref's stored row order, so it acts on the library's vectors
 * directly.  Free with tbpm_ham_destroy.  The TBPM solver benchmarks of the
 * paper ("AC", "DP") use the current operator J = i[H, x] and the density
 * operator rho_q = sum_i exp(i q.r_i)|i><i| built from the model's geometry. */
tbpm_status tbpm_build_operator(tbpm_ctx *ctx, const tbpm_ham *ref, const tbpm_csr *op, tbpm_ham **out);

/* Kubo correlation by propagation (Yuan, Roldan & Katsnelson, PRB 82, 115448;
 * PRB 84, 035439), for each of params->num_vectors random-phase vectors phi:
 *   corr[r][k] = <phi2(t_k)| A |phi1(t_k)>,  t_k = k pi / rescale, k <= N_t,
 *   phi2(t) = exp(-iHt) f(H) phi,  phi1(t) = exp(-iHt) [1 - f(H)] B phi,
 * f(E) = 1 / (1 + exp((E - mu) / kT)) applied as its Chebyshev series
 * (truncated at fermi_eps, 0: 1e-14; kT > 0).  A = op_a, B = op_b from
 * tbpm_build_operator (current operators J_alpha, J_beta for the
 * conductivity; rho_q, rho_-q for the polarization).  corr: host complex
 * [R][N_t+1].  Uses rescale, num_time_steps, num_vectors, first_vector,
 * seed, bessel_eps and lanes_per_row of params. */
tbpm_status tbpm_response_corr(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_ham *op_a, const tbpm_ham *op_b,
                               const tbpm_params *params, double mu, double kT, double fermi_eps, double *corr);
/* Host-only: Chebyshev coefficients of f(rescale x) (real), truncated after
 * the last |a_m| >= eps; TBPM_ERR_ARG if more than max_terms. */
tbpm_status tbpm_fermi_coefficients(double rescale, double mu, double kT, double eps, int32_t max_terms,
                                    double *coeff, int32_t *num_terms);
/* Host-only: real part of the AC conductivity (hbar = e = 1) from corr[N_t+1]:
 *   sigma(w) = (exp(-w/kT) - 1) / (w Omega) sum_k W_k sin(w t_k) 2 Im corr_k dt,
 * W_k = (1 + cos(pi k / N_t)) / 2, dt = pi / rescale, Omega the area (volume)
 * per orbital; omegas > 0. */
tbpm_status tbpm_ac_conductivity(const double *corr, int32_t num_time_steps, double rescale, double kT,
                                 double area_per_orbital, int32_t num_omegas, const double *omegas, double *sigma);
/* Host-only: dynamic polarization Pi(q, w) = -(2 / Omega) sum_k W_k exp(i w t_k) Im corr_k dt
 * (complex, interleaved, [num_omegas]), same grid and window. */
tbpm_status tbpm_dyn_polarization(const double *corr, int32_t num_time_steps, double rescale,
                                  double area_per_orbital, int32_t num_omegas, const double *omegas, double *pol);

/* ---- serving ------------------------------------------------------------------ */

/* A request server on `ctx`'s device: admits submitted propagations while
 * their footprints fit in hbm_budget bytes and fewer than max_slots run,
 * keeps admitted vectors resident, and advances all running requests
 * together (continuous batching).  Results do not depend on what else runs. */
tbpm_status tbpm_server_create(tbpm_ctx *ctx, size_t hbm_budget, int32_t max_slots, tbpm_server **out);
/* Queues a tbpm_propagate_dos request; never blocks on the GPU.  The server
 * copies *params (and its ldos_sites).  TBPM_ERR_TOO_LARGE if the request can
 * never fit the budget. */
tbpm_status tbpm_submit(tbpm_server *srv, const tbpm_ham *ham, const tbpm_params *params, uint64_t *ticket);
/* TBPM_PENDING while queued or running; once done returns the request's
 * status and, when it is TBPM_OK, copies into the optional host outputs
 *   corr      complex [R][N_t+1]: the per-vector correlation; corr_len is its
 *             capacity in complex entries and must be >= R (N_t+1);
 *   corr_mean complex [N_t+1]: the sample average over the R vectors, as in
 *             tbpm_propagate_dos; mean_len must be >= N_t+1,
 * with R and N_t those of the submitted request.  A capacity that is too
 * small returns TBPM_ERR_ARG before anything is written.  timings (optional,
 * double[3]): seconds of submit, admission and completion on the server's
 * clock.  A finished ticket stays readable until tbpm_server_destroy. */
tbpm_status tbpm_poll(tbpm_server *srv, uint64_t ticket, double *corr, int64_t corr_len, double *corr_mean,
                      int64_t mean_len, double *timings);
tbpm_status tbpm_cancel(tbpm_server *srv, uint64_t ticket);
/* Waits for every admitted and queued request, then frees the server. */
tbpm_status tbpm_server_destroy(tbpm_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* TBPM_H */
