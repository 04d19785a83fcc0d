// Internal declarations shared by the host library and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tbpm.h"
#include "tbpm_host.h"

namespace tbpm {

enum Kind { K_FIRST = 0, K_MID = 1, K_LAST = 2, K_MOM0 = 3, K_MOM = 4 };
enum DevFmt { F_CSR = 0, F_ELL = 1 };

// Arguments of one Chebyshev term (one application of H, fused with the
// recurrence update and the coefficient accumulation).
//   FIRST: y = scale*H x;          out = c_a * x + c_b * y
//   MID:   y = scale*H x - y;      out = out + c_a * y
//   LAST:  MID, then per-block partial sums of conj(psi0)*out and |out|^2
// Chebyshev moments (no out, no coefficients):
//   MOM0:  y = scale*H x;          partial sums of conj(x)*y and |x|^2
//   MOM:   y = scale*H x - y;      the same partial sums with the new y
// Clenshaw's backward recurrence (cl = 1; no out, psi the series' argument):
//   FIRST: y = c_a*scale*H x + c_b*x             (x = psi)
//   MID:   y = scale*H x - y + c_a*psi           (no_y: without the - y)
//   LAST:  MID, then the partial sums of conj(psi0)*y and |y|^2
// Vectors are blocks of B interleaved complex vectors: element (i, b) at i*B+b.
struct TermArgs {
    const void *rp;          // CSR row pointer (int32 or int64, see rp64)
    const int32_t *col;      // CSR [nnz] or ELL [w][ld]
    const void *val;         // complex, same layout as col
    int64_t n;
    int64_t ld;              // ELL slot stride (rows, padded)
    int32_t w;               // ELL width
    int32_t rp64;            // 1: row pointer is int64
    const void *x;
    void *y;
    void *out;
    const void *psi0;
    double scale;
    double ca_re, ca_im;
    double cb_re, cb_im;
    double *partials;        // [grid][B][4] (LAST, MOM0, MOM)
    // optional: process only the rows of the patches plist[0..pcount) of a
    // patch-reordered H (patch q: rows patch_ptr[q] .. patch_ptr[q+1]-1, at most
    // patch_tiles tiles); the other rows are left untouched
    const int32_t *plist;
    int64_t pcount;
    const int32_t *patch_ptr;
    int32_t patch_tiles;
    // Clenshaw mode (FIRST, MID, LAST kinds)
    int32_t cl;
    int32_t no_y;
    const void *psi;
    // patch-reordered H: number of patches (with patch_ptr), patch-local
    // columns [w][ld] and the halo lists, for the kernel that stages each
    // patch's x in LDS (KernelShape::staged)
    int64_t npatch;
    const uint64_t *lcol;
    const int32_t *halo_ptr, *halo_rows;
    // value table (staged kernel; null: values from val): one-byte indices,
    // four slots a word [(w+3)/4][ld]; the table [256]; per-row diagonal
    // values for index 255 (null when the table holds the diagonal)
    const uint32_t *vidx;
    const void *vtab;
    const void *vdiag;
    int32_t vdiag_real;      // vdiag holds real parts only (double or float)
};

struct KernelShape {
    int B;       // vectors per block
    int lr;      // lanes per row (B == 1: lanes splitting a row; B > 1: B, or B/2 for
                 // complex64, where a lane owns two vectors)
    int grid;    // workgroups (multiple of 8); with `staged`, the number of partial-sum
                 // blocks (staged_blocks: one per run of rows of a patch)
    int staged;  // complex64 block on patch-reordered H: the patch's x staged in LDS
};
// whether the staged complex64 SpMM kernel covers a block of B vectors on a
// patch-reordered ELL of width w with patches of at most patch_rows rows
bool staged_supported(int dtype, int B, int w, int patch_rows);
// workgroups (and partial-sum blocks) of the staged kernel for npatch patches
int staged_blocks(int B, int64_t npatch);
// lanes per row of a block of B > 1 vectors in precision dtype
inline int block_lanes(int B, int dtype) { return dtype == TBPM_C64 ? B / 2 : B; }

// launchers (tbpm_kernels.hip); all return hipSuccess or the launch error
hipError_t launch_term(int kind, int dtype, int fmt, const TermArgs &a, const KernelShape &s, hipStream_t st);
// perm (nullable): original row index of each stored row
hipError_t launch_init_random(int dtype, void *psi0, void *p, int64_t n, int B, uint64_t seed, int64_t r0,
                              const int32_t *perm, hipStream_t st);
hipError_t launch_pack_states(int dtype, const double *src, void *psi0, void *p, int64_t n, int B,
                              const int32_t *perm, hipStream_t st);
// site-localised states: vector b of the block is 1 at stored row rows[b], 0 elsewhere
struct SiteRows {
    int64_t r[64];
};
hipError_t launch_init_sites(int dtype, void *psi0, void *p, int64_t n, int B, const SiteRows &rows, hipStream_t st);
hipError_t launch_unpack_state(int dtype, const void *src, double *dst, int64_t n, int B, int b,
                               const int32_t *perm, hipStream_t st);

// Two Chebyshev terms in one pass (patch-reordered ELL, one vector):
//   y_m     = scale H x_{m-1} - y_{m-2}   (into yout, kept on chip for the patch + halo)
//   x_{m+1} = scale H y_m - x_{m-1}       (into xout)
//   out    += c_m y_m + c_{m+1} x_{m+1}   (LAST: + per-patch correlation partial sums)
struct PairArgs {
    const uint64_t *lcol;    // patch-local column indices, 4 to a word [(w+3)/4][ld]: < cnt in the patch, else cnt + halo position
    const void *val;
    int64_t ld;
    int32_t w;
    int64_t n;
    int64_t npatch;
    const int32_t *patch_ptr, *halo_ptr, *halo_rows;
    const int32_t *hcol;     // halo rows' H, contiguous per patch: slot s of halo entry g at s*ldh + g
    const void *hval;
    int64_t ldh;
    const void *xin, *yin;
    void *yout, *xout, *out;
    const void *psi0;
    double scale;
    double c0_re, c0_im, c1_re, c1_im;
    double c2_re, c2_im;     // FIRST, CROSS: the third coefficient
    void *out2;              // CROSS: the next step's accumulated series
    double *partials;        // [npatch][4]
    double *partials2;       // PAIR_MOM: the second term's [npatch][4]
    // optional: only the patches plist[0..pcount) (partials still indexed by patch)
    const int32_t *plist;
    int64_t pcount;
    // Clenshaw modes: psi (the series' argument vector), the factor ka of the
    // first product and of x in the second phase (CL_FIRST), and the second
    // phase's scale
    const void *psi;
    double ka_re, ka_im;
    double scale_b;
    // value table (null vidx: values from val and hval): index words of the
    // rows [(w+3)/4][ld] and of the halo copy [(w+3)/4][ldh], the table [256],
    // per-row diagonal values (index 255) or null
    const uint32_t *vidx, *hvidx;
    const void *vtab;
    const void *vdiag;
    int32_t vdiag_real;      // vdiag holds real parts only (double or float)
    // complex64 blocks (bpair_kernel): B = 8 or 16 vectors, modes MID and LAST
    // (partials [npatch][B][4]); 0 or 1: one vector.  max_halo: the largest
    // halo of a patch, in rows
    int32_t B;
    int32_t max_halo;
};
// pair modes: MID, LAST (+ correlation partials), MOM (moments: no out; with
// x = xin = p_m, partials = (<x|y>, <x|x>) and partials2 = (<y|z>, <y|y>) for
// y = yout = p_m+1 and z = xout = p_m+2).
// Clenshaw modes, for O = sum_m c_m T_m(H/rho) psi by the backward recurrence
// b_m = c_m psi + (2/rho) H b_m+1 - b_m+2, O = c_0 psi + (1/rho) H b_1 - b_2:
//   CL:        y = scale H x - yin + c0 psi (patch rows to yout, halo rows to
//              LDS); x' = scale_b H y - x + c1 psi (to xout);
//   CL_FIRST:  the same with xin = psi = b_{M-1} / c_{M-1} and no yin:
//              y = ka scale H x + c0 psi, x' = scale_b H y - ka x + c1 psi;
//   CL_LAST:   CL with dots: y = b_1 stays in LDS, x' = O (scale_b = 1/rho)
//              to xout, partials <psi0|O>, <O|O>;
//   CL_SINGLE: the first phase of CL only, for patch rows (yout may equal yin).
// Forward modes that straddle time steps (one vector, dots):
//   FIRST: terms 1 and 2 of a step from psi = xin (no yin, no out read):
//          y = p_1 = scale H psi; x' = p_2 = scale_b H p_1 - psi;
//          out = c0 psi + c1 p_1 + c2 p_2 (written, not read);
//   CROSS: the last term of a step and term 1 of the next:
//          psi' = out + c0 (scale H x - yin) for patch and halo rows (to yout
//          for the patch rows, kept in LDS); x' = p_1' = scale_b H psi' (to
//          xout); out2 = c1 psi' + c2 p_1'; partials of <psi0|psi'>, <psi'|psi'>.
enum PairMode { PAIR_MID = 0, PAIR_LAST = 1, PAIR_MOM = 2, PAIR_CL = 3, PAIR_CL_LAST = 4, PAIR_CL_SINGLE = 5,
                PAIR_CL_FIRST = 6, PAIR_FIRST = 7, PAIR_CROSS = 8 };
constexpr int PAIR_WG = 1024;        // lanes per workgroup of the pair kernel
// halo rows a patch may have: LDS holds y_m for (patch + halo) rows
constexpr int pair_halo_max(int patch_rows) { return patch_rows > PAIR_WG ? 1024 : 2048; }
bool pair_supported(int w, int patch_rows);
// fused pairs of complex64 blocks: B of 8 or 16, patches of at most 1024 rows
// with halos of at most 1280 rows
bool bpair_supported(int dtype, int B, int w, int patch_rows, int max_halo);

hipError_t launch_pair(int mode, int dtype, const PairArgs &a, int patch_rows, hipStream_t st);
int pair_grid(int64_t npatch);
hipError_t launch_halo_ell(int dtype, const int32_t *col, const void *val, int64_t ld, int32_t w,
                           const int32_t *halo_rows, int64_t nhalo, int64_t ldh, int32_t *hcol, void *hval,
                           hipStream_t st);
// patch-local column indices (uint16, same [w][ld] layout as col) of a
// patch-reordered ELL, for the fused pair kernel; *bad (device) is or-ed with 1
// when a column lies outside its row's patch and halo
hipError_t launch_value_index(int dtype, const int32_t *col, const void *val, int64_t n, int32_t w, int64_t ld,
                              const uint64_t *keys, int32_t nkeys, int32_t diag, uint32_t *vidx, void *vdiag,
                              int32_t *bad, hipStream_t st);   // diag: 0 none, 1 complex, 2 real parts
hipError_t launch_halo_vidx(const uint32_t *vidx, int64_t ld, int32_t nw, const int32_t *halo_rows, int64_t nhalo,
                            int64_t ldh, uint32_t *hvidx, hipStream_t st);
hipError_t launch_local_cols(const int32_t *col, int64_t ld, int32_t w, int64_t n, const int32_t *patch_ptr,
                             int64_t npatch, const int32_t *halo_ptr, const int32_t *halo_rows, uint64_t *lcol,
                             int32_t *bad, hipStream_t st);
hipError_t launch_to_ell_perm(int dtype, const int64_t *rp, const int32_t *col, const double *val, int64_t n,
                              int32_t w, int64_t ld, const int32_t *old_of_new, const int32_t *new_of_old,
                              int32_t *col_out, void *val_out, hipStream_t st);
hipError_t launch_dot_partials(int dtype, const void *psi0, const void *v, int64_t n, int B, double *partials,
                               int grid, hipStream_t st);
// tol > 0 and flag: *flag (device) is set to 1 when some |norm - 1| > tol
hipError_t launch_reduce(const double *partials, int nblocks, int B, double *corr, double *norms,
                         hipStream_t st, double tol = 0.0, int32_t *flag = nullptr);
// as launch_reduce, with the step index k read from *kstep (device) and
// advanced by one: corr[k][b], norms[k][b] for rows of B (graph-replayable)
hipError_t launch_reduce_step(const double *partials, int nblocks, int B, double *corr, double *norms, int32_t *kstep,
                              hipStream_t st, double tol = 0.0, int32_t *flag = nullptr);
hipError_t launch_set_counter(int32_t *counter, int32_t value, hipStream_t st);
// moments: partials of `count` consecutive MOM0/MOM launches (launch j at
// partials + j * stride, [nblocks][B][4]) summed in a fixed order into
// raw[b][m0 + j][0..2] = (Re, Im of <p_j|p_{j+1}>, <p_j|p_j>), raw row length kmax
hipError_t launch_moment_reduce(const double *partials, int nblocks, int B, int64_t stride, int count, int m0,
                                double *raw, int kmax, hipStream_t st);
// mu[b][q], q < num: mu_2m = 2<p_m|p_m> - mu_0, mu_2m+1 = 2<p_m|p_m+1> - mu_1
hipError_t launch_moment_finish(const double *raw, int kmax, int B, int num, double *mu, hipStream_t st);
hipError_t launch_ldos_gather(int dtype, const void *psi0, const void *v, int64_t n, int B,
                              const int64_t *sites, int nsites, double *site_corr, int stride, int k,
                              hipStream_t st);
// operators stored as CSR in H's row order (tbpm_build_operator), one vector:
//   op_apply: y = A x
//   op_dot:   partials[blk][0..1] = sum over the rows of workgroup blk of conj(u_i) (A v)_i
//             (fixed order; partials[blk][2..3] = 0), grid = op_dot_grid(n) <= 1024
hipError_t launch_op_apply(int dtype, const void *rp, int rp64, const int32_t *col, const void *val, int64_t n,
                           const void *x, void *y, hipStream_t st);
hipError_t launch_op_dot(int dtype, const void *rp, int rp64, const int32_t *col, const void *val, int64_t n,
                         const void *u, const void *v, double *partials, hipStream_t st);
int op_dot_grid(int64_t n);
// quasi-eigenstates: qe[j][i] += f_j psi[i] for j < count (<= QE_MAX), psi one
// vector in storage precision, qe complex128 [count][n]
constexpr int QE_MAX = 16;
struct QeFactors {
    double re[QE_MAX], im[QE_MAX];
};
hipError_t launch_qe_accumulate(int dtype, const void *psi, int64_t n, double *qe, int count, const QeFactors &f,
                                hipStream_t st);
// analysis / conversion of an uploaded CSR (int64 row_ptr, int32 col, c128 val)
hipError_t launch_csr_check(const int64_t *rp, const int32_t *col, const double *val, int64_t n, int64_t nnz,
                            unsigned long long *res /*[4]: flags, maxrow, gersh bits, maxabs bits*/,
                            hipStream_t st);
hipError_t launch_hermitian_check(const int64_t *rp, const int32_t *col, const double *val, int64_t n,
                                  double tol, unsigned long long *res, hipStream_t st);
hipError_t launch_to_csr(int dtype, const int64_t *rp, const int32_t *col, const double *val, int64_t n,
                         int64_t nnz, void *rp_out, int rp64, int32_t *col_out, void *val_out, hipStream_t st);
hipError_t launch_to_ell(int dtype, const int64_t *rp, const int32_t *col, const double *val, int64_t n,
                         int32_t w, int64_t ld, int32_t *col_out, void *val_out, hipStream_t st);
// grid size (multiple of 8) for a term kernel over n rows
int term_grid(int64_t n, const KernelShape &s, int num_cu);
int rows_per_tile(const KernelShape &s);

// allocation-free propagation (tbpm_noalloc.hip): with `device` current, looks
// up the device address of the file-scope scratch area on it (once per device)
hipError_t noalloc_init(int device);

}  // namespace tbpm

// ---- opaque objects ----------------------------------------------------------

struct tbpm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    tbpm_allocator alloc{};
    bool has_alloc = false;
    int num_cu = 256;
    std::string last_error;
    // kernel timing (tbpm_ctx_set_profiling): per kind first / middle / last term
    bool profiling = false;
    double kernel_ms[3] = {0, 0, 0};
    int64_t kernel_launches[3] = {0, 0, 0};
    std::vector<hipEvent_t> events;   // reusable pool
    // time steps captured in HIP graphs: 0 never, 1 small problems, 2 whenever possible
    int graphs = 1;
    std::atomic<int64_t> graph_replays{0};   // also advanced by the server's thread
    // series evaluation (TBPM_SERIES_*); read when a job starts, also by the server's thread
    std::atomic<int> series{TBPM_SERIES_FORWARD};
    // result of setting up the allocation-free scratch area on this device
    hipError_t noalloc_status = hipSuccess;
    void *dev_alloc(size_t bytes);
    void dev_free(void *p);
};

struct tbpm_ham {
    tbpm_ctx *ctx = nullptr;
    int64_t n = 0, nnz = 0;
    int32_t dtype = TBPM_C128;
    int32_t format = TBPM_FMT_CSR;
    double gersh = 0.0;
    double maxabs = 0.0;
    int32_t max_row = 0;
    size_t bytes = 0;
    // CSR
    void *rp = nullptr;
    int32_t rp64 = 0;
    int32_t *col = nullptr;
    void *val = nullptr;
    // ELL
    int32_t ell_w = 0;
    int64_t ell_ld = 0;
    // lanes per row for single-vector CSR terms; tuned block width (0: none)
    int lpr = 4;
    int tuned_block = 0;
    // patch reordering (TBPM_FMT_PATCH): rows renumbered; ELL holds H' = P H P^T
    bool patched = false;
    int patch_rows = 0;                 // rows per patch (workgroup size x rows per lane)
    int64_t npatch = 0;
    int32_t *patch_ptr = nullptr;       // device [npatch+1]
    int32_t *halo_ptr = nullptr;        // device [npatch+1]
    int32_t *halo_rows = nullptr;       // device [total halo]
    int32_t *old_of_new = nullptr;      // device [n]
    uint64_t *lcol = nullptr;           // device [(w+3)/4][ld]: patch-local column indices, 4 to a word
    int32_t *hcol = nullptr;            // device [w][ldh]: H rows of every patch's halo, in halo order
    void *hval = nullptr;
    int64_t ldh = 0;
    // value table of the patch format (ValueTable): vidx [(w+3)/4][ld] index
    // words, hvidx the same for the halo copy, vtab [256] values, vdiag [n]
    // diagonal values (index 255) or null; table_size 0 when not used
    uint32_t *vidx = nullptr;
    uint32_t *hvidx = nullptr;
    void *vtab = nullptr;
    void *vdiag = nullptr;
    int32_t vdiag_real = 0;             // vdiag holds the real parts only (imaginary parts all +0)
    int32_t table_size = 0;
    std::vector<int32_t> new_of_old;    // host [n]
    // host copies for the light cone of site-localised states: patch bounds
    // [npatch+1], and the stored ELL columns [w][ld] (fetched on first use)
    std::vector<int32_t> h_patch_ptr;
    mutable std::vector<int32_t> h_ell_col;
    mutable std::mutex host_mu;
    double halo_fraction = 0.0;
    int32_t max_halo = 0;               // largest halo of a patch, in rows
    mutable std::atomic<int> users{0};   // queued or running requests using this H
};
