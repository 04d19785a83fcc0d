// C ABI of the TBPM library: contexts, Hamiltonians, synchronous propagation
// and the host-side DOS transform.  The request server is in tbpm_server.cpp.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "tbpm_engine.h"
#include "tbpm_patch.h"
#include "tbpm_trace.h"

using namespace tbpm;

#define CTX_HIP(ctx, expr)                                                                    \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) {                                                               \
            (ctx)->last_error = std::string(#expr) + ": " + hipGetErrorString(e_);           \
            return TBPM_ERR_HIP;                                                              \
        }                                                                                     \
    } while (0)

static tbpm_status set_err(tbpm_ctx *ctx, tbpm_status s, const std::string &msg)
{
    if (ctx)
        ctx->last_error = msg;
    return s;
}

void *tbpm_ctx::dev_alloc(size_t bytes)
{
    if (bytes == 0)
        bytes = 256;
    if (has_alloc)
        return alloc.alloc(bytes, alloc.user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess)
        return nullptr;
    return p;
}

void tbpm_ctx::dev_free(void *p)
{
    if (!p)
        return;
    if (has_alloc)
        alloc.free(p, alloc.user);
    else
        (void)hipFree(p);
}

extern "C" {


const char *tbpm_last_error(const tbpm_ctx *ctx)
{
    if (!ctx)
        return "null context";
    return ctx->last_error.c_str();
}

tbpm_status tbpm_ctx_create(int device, const tbpm_allocator *alloc, void *hip_stream, tbpm_ctx **out)
{
    if (!out)
        return TBPM_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return TBPM_ERR_HIP;
    if (device < 0 || device >= count)
        return TBPM_ERR_ARG;
    if (alloc && (!alloc->alloc || !alloc->free))
        return TBPM_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess)
        return TBPM_ERR_HIP;
    tbpm_ctx *ctx = new (std::nothrow) tbpm_ctx();
    if (!ctx)
        return TBPM_ERR_OOM;
    ctx->device = device;
    if (alloc) {
        ctx->alloc = *alloc;
        ctx->has_alloc = true;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->num_cu = prop.multiProcessorCount;
    // the allocation-free entry point's scratch area on this device (checked there)
    ctx->noalloc_status = tbpm::noalloc_init(device);
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return TBPM_ERR_HIP;
        }
        ctx->own_stream = true;
    }
    *out = ctx;
    return TBPM_OK;
}

tbpm_status tbpm_ctx_set_profiling(tbpm_ctx *ctx, int32_t enable)
{
    if (!ctx)
        return TBPM_ERR_ARG;
    ctx->profiling = enable != 0;
    if (ctx->profiling)
        for (int k = 0; k < 3; ++k) {
            ctx->kernel_ms[k] = 0.0;
            ctx->kernel_launches[k] = 0;
        }
    return TBPM_OK;
}

tbpm_status tbpm_ctx_set_graphs(tbpm_ctx *ctx, int32_t mode)
{
    if (!ctx || mode < 0 || mode > 2)
        return TBPM_ERR_ARG;
    ctx->graphs = mode;
    return TBPM_OK;
}

tbpm_status tbpm_ctx_set_series(tbpm_ctx *ctx, int32_t mode)
{
    if (!ctx || (mode != TBPM_SERIES_FORWARD && mode != TBPM_SERIES_CLENSHAW))
        return TBPM_ERR_ARG;
    ctx->series = mode;
    return TBPM_OK;
}

tbpm_status tbpm_ctx_graph_replays(const tbpm_ctx *ctx, int64_t *replays)
{
    if (!ctx || !replays)
        return TBPM_ERR_ARG;
    *replays = ctx->graph_replays.load();
    return TBPM_OK;
}

tbpm_status tbpm_ctx_kernel_time(const tbpm_ctx *ctx, int32_t kind, double *total_ms, int64_t *launches)
{
    if (!ctx || kind < 0 || kind > 2)
        return TBPM_ERR_ARG;
    if (total_ms)
        *total_ms = ctx->kernel_ms[kind];
    if (launches)
        *launches = ctx->kernel_launches[kind];
    return TBPM_OK;
}

tbpm_status tbpm_ctx_destroy(tbpm_ctx *ctx)
{
    if (!ctx)
        return TBPM_ERR_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->events)
        (void)hipEventDestroy(e);
    if (ctx->own_stream)
        (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return TBPM_OK;
}


// nearest power of two (in log scale) to the mean row length, 1..16
static int lanes_per_row(double avg)
{
    int best = 1;
    double bd = 1e300;
    for (int l = 1; l <= 16; l *= 2) {
        const double d = std::fabs(std::log(avg > 0.5 ? avg : 0.5) - std::log((double)l));
        if (d < bd) {
            bd = d;
            best = l;
        }
    }
    return best;
}

// Stores the value table of a patch-format H (after its ELL and halo copy):
// the index words of the rows and of the halo copy, the 256-entry table, and
// the per-row diagonal values when the table leaves the diagonal out.
static hipError_t store_value_table(tbpm_ham *ham, const tbpm::ValueTable &vt, int64_t nh, hipStream_t st)
{
    tbpm_ctx *ctx = ham->ctx;
    const size_t vsz = ham->dtype == TBPM_C128 ? 16 : 8;
    const int nkeys = (int)(vt.keys.size() / 2);
    const int nw = (ham->ell_w + 3) / 4;
    const int64_t ldh = std::max<int64_t>(ham->ldh, 256);
    ham->vidx = (uint32_t *)ctx->dev_alloc((size_t)nw * (size_t)ham->ell_ld * 4);
    ham->hvidx = (uint32_t *)ctx->dev_alloc((size_t)nw * (size_t)ldh * 4);
    ham->vtab = ctx->dev_alloc(256 * vsz);
    if (vt.diag)
        ham->vdiag = ctx->dev_alloc((size_t)ham->n * (vt.diag_real ? vsz / 2 : vsz));
    uint64_t *d_keys = (uint64_t *)ctx->dev_alloc(vt.keys.size() * 8);
    int32_t *d_bad = (int32_t *)ctx->dev_alloc(256);
    // the table's values from the keys' bit patterns, zeros past the last entry
    std::vector<unsigned char> tab(256 * vsz, 0);
    for (int q = 0; q < nkeys; ++q) {
        if (vsz == 16) {
            std::memcpy(&tab[q * 16], &vt.keys[2 * q], 8);
            std::memcpy(&tab[q * 16 + 8], &vt.keys[2 * q + 1], 8);
        } else {
            const uint32_t re = (uint32_t)vt.keys[2 * q], im = (uint32_t)vt.keys[2 * q + 1];
            std::memcpy(&tab[q * 8], &re, 4);
            std::memcpy(&tab[q * 8 + 4], &im, 4);
        }
    }
    hipError_t e = hipSuccess;
    if (!ham->vidx || !ham->hvidx || !ham->vtab || (vt.diag && !ham->vdiag) || !d_keys || !d_bad)
        e = hipErrorOutOfMemory;
    if (e == hipSuccess)
        e = hipMemsetAsync(ham->vidx, 0, (size_t)nw * (size_t)ham->ell_ld * 4, st);
    if (e == hipSuccess)
        e = hipMemsetAsync(ham->hvidx, 0, (size_t)nw * (size_t)ldh * 4, st);
    if (e == hipSuccess)
        e = hipMemsetAsync(d_bad, 0, 4, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_keys, vt.keys.data(), vt.keys.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ham->vtab, tab.data(), tab.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_value_index(ham->dtype, ham->col, ham->val, ham->n, ham->ell_w, ham->ell_ld, d_keys, nkeys,
                               vt.diag ? (vt.diag_real ? 2 : 1) : 0, ham->vidx, ham->vdiag, d_bad, st);
    if (e == hipSuccess)
        e = launch_halo_vidx(ham->vidx, ham->ell_ld, nw, ham->halo_rows, nh, ham->ldh, ham->hvidx, st);
    int32_t bad = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&bad, d_bad, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    ctx->dev_free(d_keys);
    ctx->dev_free(d_bad);
    if (e == hipSuccess && bad != 0)
        e = hipErrorInvalidValue;                   // a stored value missing from the table: a planner bug
    if (e != hipSuccess) {
        ctx->dev_free(ham->vidx);
        ctx->dev_free(ham->hvidx);
        ctx->dev_free(ham->vtab);
        ctx->dev_free(ham->vdiag);
        ham->vidx = ham->hvidx = nullptr;
        ham->vtab = ham->vdiag = nullptr;
        return e;
    }
    ham->table_size = nkeys;
    ham->vdiag_real = vt.diag && vt.diag_real ? 1 : 0;
    return hipSuccess;
}

tbpm_status tbpm_build_csr(tbpm_ctx *ctx, const tbpm_csr *csr, int32_t dtype, int32_t format, int32_t flags,
                           tbpm_ham **out)
{
    if (!ctx)
        return TBPM_ERR_ARG;
    if (!csr || !out)
        return set_err(ctx, TBPM_ERR_ARG, "csr and out must not be NULL");
    *out = nullptr;
    if (dtype != TBPM_C128 && dtype != TBPM_C64)
        return set_err(ctx, TBPM_ERR_ARG, "dtype must be TBPM_C128 or TBPM_C64");
    if (format != TBPM_FMT_CSR && format != TBPM_FMT_ELL && format != TBPM_FMT_AUTO && format != TBPM_FMT_PATCH)
        return set_err(ctx, TBPM_ERR_ARG, "unknown format");
    TraceRange range("tbpm_build_csr");
    const int64_t n = csr->n, nnz = csr->nnz;
    if (n < 1 || n > INT32_MAX || nnz < 0)
        return set_err(ctx, TBPM_ERR_ARG, "n must be in [1, 2^31) and nnz >= 0");
    if (!csr->row_ptr || (nnz > 0 && (!csr->col || !csr->val)))
        return set_err(ctx, TBPM_ERR_ARG, "CSR arrays must not be NULL");
    CTX_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;

    // stage the input on the device as (int64 row_ptr, int32 col, complex128 val)
    const int64_t *d_rp = csr->row_ptr;
    const int32_t *d_col = csr->col;
    const double *d_val = csr->val;
    void *s_rp = nullptr, *s_col = nullptr, *s_val = nullptr;
    unsigned long long *d_res = nullptr;
    auto cleanup = [&]() {
        ctx->dev_free(s_rp);
        ctx->dev_free(s_col);
        ctx->dev_free(s_val);
        ctx->dev_free(d_res);
    };
    if (!csr->on_device) {
        s_rp = ctx->dev_alloc((size_t)(n + 1) * 8);
        s_col = ctx->dev_alloc((size_t)std::max<int64_t>(nnz, 1) * 4);
        s_val = ctx->dev_alloc((size_t)std::max<int64_t>(nnz, 1) * 16);
        if (!s_rp || !s_col || !s_val) {
            cleanup();
            return set_err(ctx, TBPM_ERR_OOM, "device allocation of the CSR staging buffers failed");
        }
        hipError_t e = hipMemcpyAsync(s_rp, csr->row_ptr, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && nnz > 0)
            e = hipMemcpyAsync(s_col, csr->col, (size_t)nnz * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && nnz > 0)
            e = hipMemcpyAsync(s_val, csr->val, (size_t)nnz * 16, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            cleanup();
            return set_err(ctx, TBPM_ERR_HIP, std::string("CSR upload: ") + hipGetErrorString(e));
        }
        d_rp = (const int64_t *)s_rp;
        d_col = (const int32_t *)s_col;
        d_val = (const double *)s_val;
    }
    d_res = (unsigned long long *)ctx->dev_alloc(4 * sizeof(unsigned long long));
    if (!d_res) {
        cleanup();
        return set_err(ctx, TBPM_ERR_OOM, "device allocation failed");
    }
    unsigned long long res[4] = {0, 0, 0, 0};
    hipError_t e = hipMemsetAsync(d_res, 0, sizeof(res), st);
    if (e == hipSuccess)
        e = launch_csr_check(d_rp, d_col, d_val, n, nnz, d_res, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(res, d_res, sizeof(res), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        cleanup();
        return set_err(ctx, TBPM_ERR_HIP, std::string("CSR check: ") + hipGetErrorString(e));
    }
    if (res[0]) {
        cleanup();
        std::string why;
        if (res[0] & 1) why += " row_ptr not monotone or not ending at nnz;";
        if (res[0] & 2) why += " column index out of range;";
        if (res[0] & 4) why += " columns not strictly increasing within a row;";
        return set_err(ctx, TBPM_ERR_CSR, "malformed CSR:" + why);
    }
    double gersh, maxabs;
    std::memcpy(&gersh, &res[2], 8);
    std::memcpy(&maxabs, &res[3], 8);
    const int32_t max_row = (int32_t)res[1];
    if (flags & TBPM_BUILD_CHECK_HERMITIAN) {
        res[0] = 0;
        e = hipMemsetAsync(d_res, 0, sizeof(res), st);
        if (e == hipSuccess)
            e = launch_hermitian_check(d_rp, d_col, d_val, n, 1e-14 * maxabs, d_res, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(res, d_res, 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            cleanup();
            return set_err(ctx, TBPM_ERR_HIP, std::string("Hermitian check: ") + hipGetErrorString(e));
        }
        if (res[0] & 8) {
            cleanup();
            return set_err(ctx, TBPM_ERR_CSR, "H is not Hermitian: some H_ij differs from conj(H_ji)");
        }
    }

    tbpm_ham *ham = new (std::nothrow) tbpm_ham();
    if (!ham) {
        cleanup();
        return set_err(ctx, TBPM_ERR_OOM, "host allocation failed");
    }
    ham->ctx = ctx;
    ham->n = n;
    ham->nnz = nnz;
    ham->dtype = dtype;
    ham->gersh = gersh;
    ham->maxabs = maxabs;
    ham->max_row = max_row;
    ham->lpr = lanes_per_row((double)nnz / (double)n);
    int fmt = format;
    const double pad = (double)max_row * (double)n;
    const bool ell_ok = max_row > 0 && max_row <= 64 && pad <= 1.15 * (double)nnz;
    if (fmt == TBPM_FMT_AUTO) {
        // ELL when padding costs at most 15% extra entries; patch-reordered ELL
        // (two terms per pass) for large matrices whose row length has a fused
        // kernel and whose patch halos fit on chip (else plain ELL)
        if (ell_ok && n >= 65536 && pair_supported(max_row, PAIR_WG))
            fmt = TBPM_FMT_PATCH;
        else
            fmt = ell_ok ? TBPM_FMT_ELL : TBPM_FMT_CSR;
    }
    const size_t vsz = dtype == TBPM_C128 ? 16 : 8;
    if (fmt == TBPM_FMT_PATCH) {
        // patch reordering needs the structure on the host; falls back to ELL
        // when a halo is too large or the row length has no fused kernel
        const int prow = (max_row <= 5 && (flags & TBPM_BUILD_LARGE_PATCHES)) ? 2 * PAIR_WG : PAIR_WG;
        bool ok = max_row > 0 && pair_supported(max_row, prow);
        std::vector<int64_t> h_rp;
        std::vector<int32_t> h_col;
        const int64_t *hrp = csr->row_ptr;
        const int32_t *hcol = csr->col;
        if (ok && csr->on_device) {
            h_rp.resize((size_t)n + 1);
            h_col.resize((size_t)std::max<int64_t>(nnz, 1));
            e = hipMemcpy(h_rp.data(), d_rp, (size_t)(n + 1) * 8, hipMemcpyDeviceToHost);
            if (e == hipSuccess && nnz > 0)
                e = hipMemcpy(h_col.data(), d_col, (size_t)nnz * 4, hipMemcpyDeviceToHost);
            if (e != hipSuccess) {
                tbpm_ham_destroy(ham);
                cleanup();
                return set_err(ctx, TBPM_ERR_HIP, std::string("CSR download: ") + hipGetErrorString(e));
            }
            hrp = h_rp.data();
            hcol = h_col.data();
        }
        tbpm::PatchPlan plan;
        if (ok)
            ok = tbpm::plan_patches(n, hrp, hcol, prow, pair_halo_max(prow), plan);
        if (ok) {
            const int64_t np = (int64_t)plan.patch_ptr.size() - 1;
            std::vector<int32_t> hp32(plan.halo_ptr.begin(), plan.halo_ptr.end());
            ham->npatch = np;
            ham->patch_rows = prow;
            ham->halo_fraction = plan.halo_fraction;
            ham->max_halo = plan.max_halo;
            ham->h_patch_ptr = plan.patch_ptr;
            ham->patch_ptr = (int32_t *)ctx->dev_alloc((size_t)(np + 1) * 4);
            ham->halo_ptr = (int32_t *)ctx->dev_alloc((size_t)(np + 1) * 4);
            ham->halo_rows = (int32_t *)ctx->dev_alloc(std::max<size_t>(plan.halo_rows.size(), 1) * 4);
            ham->old_of_new = (int32_t *)ctx->dev_alloc((size_t)n * 4);
            int32_t *d_new = (int32_t *)ctx->dev_alloc((size_t)n * 4);
            ham->ell_w = max_row;
            ham->ell_ld = (n + 255) / 256 * 256;
            const size_t slots = (size_t)ham->ell_w * (size_t)ham->ell_ld;
            ham->col = (int32_t *)ctx->dev_alloc(slots * 4);
            ham->val = ctx->dev_alloc(slots * vsz);
            if (!ham->patch_ptr || !ham->halo_ptr || !ham->halo_rows || !ham->old_of_new || !d_new || !ham->col ||
                !ham->val) {
                ctx->dev_free(d_new);
                tbpm_ham_destroy(ham);
                cleanup();
                return set_err(ctx, TBPM_ERR_OOM, "device allocation of the reordered H failed");
            }
            e = hipMemcpyAsync(ham->patch_ptr, plan.patch_ptr.data(), (size_t)(np + 1) * 4, hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(ham->halo_ptr, hp32.data(), (size_t)(np + 1) * 4, hipMemcpyHostToDevice, st);
            if (e == hipSuccess && !plan.halo_rows.empty())
                e = hipMemcpyAsync(ham->halo_rows, plan.halo_rows.data(), plan.halo_rows.size() * 4,
                                   hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(ham->old_of_new, plan.old_of_new.data(), (size_t)n * 4, hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpyAsync(d_new, plan.new_of_old.data(), (size_t)n * 4, hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = launch_to_ell_perm(dtype, d_rp, d_col, d_val, n, ham->ell_w, ham->ell_ld, ham->old_of_new, d_new,
                                       ham->col, ham->val, st);
            // patch-local 16-bit column indices for the fused pairs
            int32_t *d_bad = nullptr;
            if (e == hipSuccess) {
                ham->lcol = (uint64_t *)ctx->dev_alloc((size_t)((ham->ell_w + 3) / 4) * (size_t)ham->ell_ld * 8);
                d_bad = (int32_t *)ctx->dev_alloc(256);
                if (!ham->lcol || !d_bad)
                    e = hipErrorOutOfMemory;
            }
            if (e == hipSuccess)
                e = hipMemsetAsync(d_bad, 0, 4, st);
            if (e == hipSuccess)
                e = launch_local_cols(ham->col, ham->ell_ld, ham->ell_w, n, ham->patch_ptr, np, ham->halo_ptr,
                                      ham->halo_rows, ham->lcol, d_bad, st);
            int32_t bad = 0;
            if (e == hipSuccess)
                e = hipMemcpyAsync(&bad, d_bad, 4, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess)
                e = hipStreamSynchronize(st);
            ctx->dev_free(d_bad);
            if (e == hipSuccess && bad != 0)
                e = hipErrorInvalidValue;           // a column outside its patch and halo: a planner bug
            // contiguous copy of each patch's halo rows of H'
            const int64_t nh = (int64_t)plan.halo_rows.size();
            ham->ldh = (nh + 255) / 256 * 256;
            if (e == hipSuccess) {
                ham->hcol = (int32_t *)ctx->dev_alloc((size_t)ham->ell_w * std::max<int64_t>(ham->ldh, 256) * 4);
                ham->hval = ctx->dev_alloc((size_t)ham->ell_w * std::max<int64_t>(ham->ldh, 256) * vsz);
                if (!ham->hcol || !ham->hval)
                    e = hipErrorOutOfMemory;
            }
            if (e == hipSuccess)
                e = launch_halo_ell(dtype, ham->col, ham->val, ham->ell_ld, ham->ell_w, ham->halo_rows, nh, ham->ldh,
                                    ham->hcol, ham->hval, st);
            // value table: one byte per entry when the hoppings take few values
            tbpm::ValueTable vt;
            if (e == hipSuccess && !csr->on_device && !(flags & TBPM_BUILD_NO_VALUE_TABLE) &&
                tbpm::plan_value_table(n, csr->row_ptr, csr->col, csr->val, dtype, vt))
                e = store_value_table(ham, vt, nh, st);
            if (e == hipSuccess)
                e = hipStreamSynchronize(st);       // host plan vectors are freed below
            ctx->dev_free(d_new);
            ham->new_of_old = std::move(plan.new_of_old);
            ham->patched = true;
            ham->format = TBPM_FMT_PATCH;
            ham->bytes = slots * (4 + vsz) + (size_t)((ham->ell_w + 3) / 4) * (size_t)ham->ell_ld * 8 +
                         (size_t)(np + 1) * 8 + plan.halo_rows.size() * 4 + (size_t)n * 4 +
                         (size_t)ham->ell_w * (size_t)ham->ldh * (4 + vsz);
            if (ham->table_size > 0)
                ham->bytes += (size_t)((ham->ell_w + 3) / 4) * (size_t)(ham->ell_ld + ham->ldh) * 4 + 256 * vsz +
                              (ham->vdiag ? (size_t)n * (ham->vdiag_real ? vsz / 2 : vsz) : 0);
        } else {
            fmt = ell_ok ? TBPM_FMT_ELL : TBPM_FMT_CSR;
        }
    }
    if (!ham->patched) {
        ham->format = fmt;
        if (fmt == TBPM_FMT_CSR) {
            ham->rp64 = nnz >= (int64_t)INT32_MAX ? 1 : 0;
            const size_t rpb = (size_t)(n + 1) * (ham->rp64 ? 8 : 4);
            ham->rp = ctx->dev_alloc(rpb);
            ham->col = (int32_t *)ctx->dev_alloc((size_t)std::max<int64_t>(nnz, 1) * 4);
            ham->val = ctx->dev_alloc((size_t)std::max<int64_t>(nnz, 1) * vsz);
            ham->bytes = rpb + (size_t)nnz * (4 + vsz);
            if (!ham->rp || !ham->col || !ham->val) {
                tbpm_ham_destroy(ham);
                cleanup();
                return set_err(ctx, TBPM_ERR_OOM, "device allocation of H failed");
            }
            e = launch_to_csr(dtype, d_rp, d_col, d_val, n, nnz, ham->rp, ham->rp64, ham->col, ham->val, st);
        } else {
            ham->ell_w = std::max(max_row, 1);
            ham->ell_ld = (n + 255) / 256 * 256;
            const size_t slots = (size_t)ham->ell_w * (size_t)ham->ell_ld;
            ham->col = (int32_t *)ctx->dev_alloc(slots * 4);
            ham->val = ctx->dev_alloc(slots * vsz);
            ham->bytes = slots * (4 + vsz);
            if (!ham->col || !ham->val) {
                tbpm_ham_destroy(ham);
                cleanup();
                return set_err(ctx, TBPM_ERR_OOM, "device allocation of H failed");
            }
            e = launch_to_ell(dtype, d_rp, d_col, d_val, n, ham->ell_w, ham->ell_ld, ham->col, ham->val, st);
        }
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    cleanup();
    if (e != hipSuccess) {
        tbpm_ham_destroy(ham);
        return set_err(ctx, TBPM_ERR_HIP, std::string("H conversion: ") + hipGetErrorString(e));
    }
    *out = ham;
    return TBPM_OK;
}

tbpm_status tbpm_ham_info(const tbpm_ham *ham, int64_t *n, int64_t *nnz, double *gershgorin, size_t *bytes,
                          int32_t *dtype, int32_t *format)
{
    if (!ham)
        return TBPM_ERR_ARG;
    if (n) *n = ham->n;
    if (nnz) *nnz = ham->nnz;
    if (gershgorin) *gershgorin = ham->gersh;
    if (bytes) *bytes = ham->bytes;
    if (dtype) *dtype = ham->dtype;
    if (format) *format = ham->format;
    return TBPM_OK;
}

tbpm_status tbpm_ham_value_table(const tbpm_ham *ham, int32_t *entries, int32_t *per_row_diagonal)
{
    if (!ham)
        return TBPM_ERR_ARG;
    if (entries) *entries = ham->table_size;
    if (per_row_diagonal) *per_row_diagonal = ham->vdiag ? (ham->vdiag_real ? 2 : 1) : 0;
    return TBPM_OK;
}

tbpm_status tbpm_ham_fused_pairs(const tbpm_ham *ham, int32_t block, int32_t *fused)
{
    if (!ham || !fused || block < 1)
        return TBPM_ERR_ARG;
    *fused = (ham->patched && (block == 1 || block_pairs(ham, block))) ? 1 : 0;
    return TBPM_OK;
}

tbpm_status tbpm_ham_destroy(tbpm_ham *ham)
{
    if (!ham)
        return TBPM_ERR_ARG;
    if (ham->users.load() > 0) {
        ham->ctx->last_error = "Hamiltonian is still used by a queued or running request";
        return TBPM_ERR_ARG;
    }
    tbpm_ctx *ctx = ham->ctx;
    (void)hipStreamSynchronize(ctx->stream);
    ctx->dev_free(ham->rp);
    ctx->dev_free(ham->col);
    ctx->dev_free(ham->val);
    ctx->dev_free(ham->patch_ptr);
    ctx->dev_free(ham->halo_ptr);
    ctx->dev_free(ham->halo_rows);
    ctx->dev_free(ham->old_of_new);
    ctx->dev_free(ham->lcol);
    ctx->dev_free(ham->hcol);
    ctx->dev_free(ham->hval);
    ctx->dev_free(ham->vidx);
    ctx->dev_free(ham->hvidx);
    ctx->dev_free(ham->vtab);
    ctx->dev_free(ham->vdiag);
    delete ham;
    return TBPM_OK;
}

tbpm_status tbpm_footprint(const tbpm_ham *ham, const tbpm_params *params, size_t *bytes)
{
    if (!ham || !params || !bytes)
        return TBPM_ERR_ARG;
    Job job;
    tbpm_status s = job.setup(ham->ctx, ham, params, nullptr);
    if (s != TBPM_OK)
        return s;
    *bytes = job.footprint();
    job.ctx = nullptr;   // nothing allocated
    return TBPM_OK;
}

// one-vector outputs of a propagation (snapshots, quasi-eigenstates)
struct Outputs {
    int32_t num_snaps = 0;
    const int32_t *snap_steps = nullptr;
    double *snaps = nullptr;
    int32_t num_energies = 0;
    const double *energies = nullptr;
    double *qe = nullptr;
};

static tbpm_status run_sync(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params, const double *psi0,
                            double *corr, double *norms, double *ldos, double *psi_final,
                            const Outputs *outs = nullptr, const int64_t *sites = nullptr, int32_t num_sites = 0,
                            double *corr_mean = nullptr)
{
    if (!ctx || !ham)
        return TBPM_ERR_ARG;
    if (ham->ctx != ctx)
        return set_err(ctx, TBPM_ERR_ARG, "Hamiltonian belongs to another context");
    if (!corr && !corr_mean)
        return set_err(ctx, TBPM_ERR_ARG, "corr (or, for tbpm_propagate_dos, corr_mean) must not be NULL");
    CTX_HIP(ctx, hipSetDevice(ctx->device));
    TraceRange range(sites ? "tbpm_propagate_sites" : outs ? "tbpm_propagate_outputs"
                     : psi0 ? "tbpm_propagate_states" : "tbpm_propagate_dos");
    Job job;
    job.given_states = psi0;
    job.final_states = psi_final;
    if (sites)
        job.site_states.assign(sites, sites + num_sites);
    if (outs) {
        job.snap_steps.assign(outs->snap_steps, outs->snap_steps + outs->num_snaps);
        job.snaps = outs->snaps;
        job.qe_energies.assign(outs->energies, outs->energies + outs->num_energies);
        job.qe_host = outs->qe;
    }
    tbpm_status s = job.setup(ctx, ham, params, ctx->stream);
    job.profile = ctx->profiling;
    if (s == TBPM_OK)
        s = job.allocate();
    if (s == TBPM_OK && job.p.norm_tol > 0.0) {
        // one block of vectors at a time, stopping after a block whose norms left
        // the tolerance (the remaining vectors' outputs stay zero)
        while ((s = job.advance(std::max(job.p.num_time_steps, 1))) == TBPM_PENDING) {
            if ((s = job.queue_flag_read()) != TBPM_OK)
                break;
            if (hipStreamSynchronize(ctx->stream) != hipSuccess || job.flag_set())
                break;
        }
        if (s == TBPM_PENDING)
            s = TBPM_OK;
    } else if (s == TBPM_OK) {
        s = job.advance(INT32_MAX);
    }
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (s == TBPM_OK && e != hipSuccess)
        return set_err(ctx, TBPM_ERR_HIP, std::string("propagation: ") + hipGetErrorString(e));
    if (s == TBPM_OK)
        s = job.collect_profile();
    if (s == TBPM_OK)
        s = job.finish(corr, norms, ldos, corr_mean);
    if (s != TBPM_OK)
        ctx->last_error = job.error;
    return s;
}

tbpm_status tbpm_propagate_dos(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params, double *corr,
                               double *norms, double *ldos_corr, double *corr_mean)
{
    return run_sync(ctx, ham, params, nullptr, corr, norms, ldos_corr, nullptr, nullptr, nullptr, 0, corr_mean);
}

tbpm_status tbpm_propagate_states(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params,
                                  const double *psi0, double *corr, double *norms, double *psi_final)
{
    if (!psi0)
        return set_err(ctx, TBPM_ERR_ARG, "psi0 must not be NULL");
    if (params && params->num_ldos_sites > 0)
        return set_err(ctx, TBPM_ERR_ARG, "per-site correlation is only defined for random-phase states");
    return run_sync(ctx, ham, params, psi0, corr, norms, nullptr, psi_final);
}

tbpm_status tbpm_propagate_sites(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params,
                                 const int64_t *sites, int32_t num_sites, double *corr, double *norms)
{
    if (!ctx)
        return TBPM_ERR_ARG;
    if (!params)
        return set_err(ctx, TBPM_ERR_ARG, "params is NULL");
    if (num_sites < 1 || !sites)
        return set_err(ctx, TBPM_ERR_ARG, "at least one site is required");
    if (params->num_ldos_sites > 0)
        return set_err(ctx, TBPM_ERR_ARG, "site-localised states take no LDOS sites");
    tbpm_params p = *params;
    p.num_vectors = num_sites;
    p.first_vector = 0;
    return run_sync(ctx, ham, &p, nullptr, corr, norms, nullptr, nullptr, nullptr, sites, num_sites);
}

tbpm_status tbpm_time_evolution(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params, const double *psi0,
                                int32_t num_snapshots, const int32_t *steps, double *snapshots, double *corr)
{
    if (!ctx)
        return TBPM_ERR_ARG;
    if (num_snapshots < 1 || !steps || !snapshots)
        return set_err(ctx, TBPM_ERR_ARG, "at least one snapshot step and its output are required");
    if (params && params->num_ldos_sites > 0)
        return set_err(ctx, TBPM_ERR_ARG, "snapshots take no LDOS sites");
    const int nt1 = params ? params->num_time_steps + 1 : 1;
    std::vector<double> scratch;
    if (!corr) {
        scratch.assign(2 * (size_t)std::max(nt1, 1), 0.0);
        corr = scratch.data();
    }
    Outputs o;
    o.num_snaps = num_snapshots;
    o.snap_steps = steps;
    o.snaps = snapshots;
    return run_sync(ctx, ham, params, psi0, corr, nullptr, nullptr, nullptr, &o);
}

tbpm_status tbpm_quasi_eigenstates(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params,
                                   const double *psi0, int32_t num_energies, const double *energies, double *qe,
                                   double *corr)
{
    if (!ctx)
        return TBPM_ERR_ARG;
    if (num_energies < 1 || !energies || !qe)
        return set_err(ctx, TBPM_ERR_ARG, "at least one energy and the output are required");
    if (params && params->num_ldos_sites > 0)
        return set_err(ctx, TBPM_ERR_ARG, "quasi-eigenstates take no LDOS sites");
    const int nt1 = params ? params->num_time_steps + 1 : 1;
    std::vector<double> scratch;
    if (!corr) {
        scratch.assign(2 * (size_t)std::max(nt1, 1), 0.0);
        corr = scratch.data();
    }
    Outputs o;
    o.num_energies = num_energies;
    o.energies = energies;
    o.qe = qe;
    return run_sync(ctx, ham, params, psi0, corr, nullptr, nullptr, nullptr, &o);
}



}  // extern "C"

// ---- autotuner ------------------------------------------------------------------------

extern "C" tbpm_status tbpm_autotune(tbpm_ctx *ctx, tbpm_ham *ham, int32_t max_block, int32_t *best_lanes,
                                     int32_t *best_block, double *us_per_vector_term)
{
    if (!ctx || !ham || ham->ctx != ctx || max_block < 1 || max_block > 64)
        return set_err(ctx, TBPM_ERR_ARG, "autotune: bad arguments");
    CTX_HIP(ctx, hipSetDevice(ctx->device));
    int bmax = 1;
    while (bmax * 2 <= max_block)
        bmax *= 2;
    const size_t elem = ham->dtype == TBPM_C128 ? 16 : 8;
    const size_t vbytes = (size_t)ham->n * bmax * elem;
    void *x = ctx->dev_alloc(vbytes), *y = ctx->dev_alloc(vbytes), *o = ctx->dev_alloc(vbytes);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        ctx->dev_free(x);
        ctx->dev_free(y);
        ctx->dev_free(o);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (!x || !y || !o) {
        release();
        return set_err(ctx, TBPM_ERR_OOM, "autotune: scratch allocation failed");
    }
    hipStream_t st = ctx->stream;
    if (hipMemsetAsync(x, 0, vbytes, st) != hipSuccess || hipMemsetAsync(y, 0, vbytes, st) != hipSuccess ||
        hipMemsetAsync(o, 0, vbytes, st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        release();
        return set_err(ctx, TBPM_ERR_HIP, "autotune: setup failed");
    }
    TermArgs a{};
    a.n = ham->n;
    if (ham->format == TBPM_FMT_CSR) {
        a.rp = ham->rp;
        a.rp64 = ham->rp64;
    } else {
        a.ld = ham->ell_ld;
        a.w = ham->ell_w;
    }
    a.col = ham->col;
    a.val = ham->val;
    a.vidx = ham->vidx;
    a.vtab = ham->vtab;
    a.vdiag = ham->vdiag;
    a.vdiag_real = ham->vdiag_real;
    a.x = x;
    a.y = y;
    a.out = o;
    a.scale = 0.0;      // scratch vectors stay zero
    const int fmt = ham->format == TBPM_FMT_CSR ? F_CSR : F_ELL;
    // time one shape: mean of 3 launches after one warm-up, microseconds
    auto time_shape = [&](KernelShape s, double *us) -> tbpm_status {
        CTX_HIP(ctx, launch_term(K_MID, ham->dtype, fmt, a, s, st));
        CTX_HIP(ctx, hipEventRecord(e0, st));
        for (int r = 0; r < 3; ++r)
            CTX_HIP(ctx, launch_term(K_MID, ham->dtype, fmt, a, s, st));
        CTX_HIP(ctx, hipEventRecord(e1, st));
        CTX_HIP(ctx, hipEventSynchronize(e1));
        float ms = 0.0f;
        CTX_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
        *us = ms * 1e3 / 3.0;
        return TBPM_OK;
    };
    int lanes = ham->lpr;
    double best1 = 1e300;
    if (ham->format == TBPM_FMT_CSR) {
        for (int l = 1; l <= 16; l *= 2) {
            KernelShape s{1, l, 0};
            s.grid = term_grid(ham->n, s, ctx->num_cu);
            double us;
            tbpm_status r = time_shape(s, &us);
            if (r != TBPM_OK) {
                release();
                return r;
            }
            if (us < best1) {
                best1 = us;
                lanes = l;
            }
        }
    } else {
        KernelShape s{1, 1, 0};
        s.grid = term_grid(ham->n, s, ctx->num_cu);
        tbpm_status r = time_shape(s, &best1);
        if (r != TBPM_OK) {
            release();
            return r;
        }
    }
    int block = 1;
    double best = best1;   // per vector
    for (int b = 2; b <= bmax; b *= 2) {
        KernelShape s{b, block_lanes(b, ham->dtype), 0};
        s.grid = term_grid(ham->n, s, ctx->num_cu);
        double us;
        tbpm_status r = time_shape(s, &us);
        if (r != TBPM_OK) {
            release();
            return r;
        }
        if (us / b < best) {
            best = us / b;
            block = b;
        }
    }
    release();
    ham->lpr = lanes;
    ham->tuned_block = block;
    if (best_lanes) *best_lanes = lanes;
    if (best_block) *best_block = block;
    if (us_per_vector_term) *us_per_vector_term = best;
    return TBPM_OK;
}

extern "C" tbpm_status tbpm_ham_set_tuning(tbpm_ham *ham, int32_t lanes_per_row, int32_t block)
{
    if (!ham)
        return TBPM_ERR_ARG;
    const bool lanes_ok = lanes_per_row == 1 || lanes_per_row == 2 || lanes_per_row == 4 || lanes_per_row == 8 ||
                          lanes_per_row == 16;
    const bool block_ok = block == 0 || (block >= 1 && block <= 64 && (block & (block - 1)) == 0);
    if (!lanes_ok || !block_ok)
        return TBPM_ERR_ARG;
    ham->lpr = lanes_per_row;
    ham->tuned_block = block;
    return TBPM_OK;
}


