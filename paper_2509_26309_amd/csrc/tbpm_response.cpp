// Response functions by propagation: AC conductivity and dynamic polarization.
//
// Both are Kubo correlations evaluated with random-phase states (Yuan,
// Roldan & Katsnelson, Phys. Rev. B 82, 115448 (2010); 84, 035439 (2011)):
//   corr(t) = <phi2(t)| A |phi1(t)>,
//   phi2(t) = exp(-iHt) f(H) phi,   phi1(t) = exp(-iHt) [1 - f(H)] B phi,
// with f the Fermi-Dirac function, A = J_alpha, B = J_beta (current
// operators) for the conductivity and A = rho_q, B = rho_-q (density
// operators) for the polarization.  f(H) is applied as its own Chebyshev
// series with the same term kernels as the time steps (real coefficients
// a_m; 1 - f(H) uses delta_m0 - a_m), and each time step of both states is
// one application of the propagator's series.  The operators are CSR
// matrices stored in H's row order (tbpm_build_operator); one fused kernel
// per step forms A phi1 and sums conj(phi2) A phi1.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "tbpm_engine.h"
#include "tbpm_trace.h"

namespace tbpm {



struct ResponseRun {
    tbpm_ctx *ctx;
    const tbpm_ham *ham;
    const tbpm_ham *opa, *opb;
    tbpm_params p;
    double mu, kT, feps;
    std::vector<double> fa, fb, coeff;   // complex interleaved
    int MF = 0, M = 0;
    size_t elem = 16;
    void *T0 = nullptr, *W = nullptr, *S1 = nullptr, *S2 = nullptr, *O = nullptr, *Q = nullptr, *X1 = nullptr,
         *X2 = nullptr;
    double *partials = nullptr, *corr_dev = nullptr, *norms_dev = nullptr;
    int max_grid = 8;
    bool pairs = false;
    bool clenshaw = false;
    KernelShape shape{};
    std::string error;

    tbpm_status fail(tbpm_status s, const std::string &m)
    {
        error = m;
        return s;
    }

    tbpm_status setup()
    {
        if (!(p.rescale > 0.0) || !std::isfinite(p.rescale))
            return fail(TBPM_ERR_ARG, "rescale must be positive");
        if (p.num_time_steps < 0)
            return fail(TBPM_ERR_ARG, "num_time_steps must be >= 0");
        if (p.num_vectors < 1 || p.first_vector < 0)
            return fail(TBPM_ERR_ARG, "num_vectors must be >= 1 and first_vector >= 0");
        if (p.num_ldos_sites != 0)
            return fail(TBPM_ERR_ARG, "response functions take no LDOS sites");
        if (!(kT > 0.0) || !std::isfinite(kT) || !std::isfinite(mu))
            return fail(TBPM_ERR_ARG, "kT must be positive and mu finite");
        for (const tbpm_ham *op : {opa, opb}) {
            if (!op || op->ctx != ctx || op->n != ham->n || op->dtype != ham->dtype || op->format != TBPM_FMT_CSR)
                return fail(TBPM_ERR_ARG, "operators must come from tbpm_build_operator on this Hamiltonian");
        }
        if (p.rescale < ham->gersh)
            return fail(TBPM_ERR_RESCALE, "rescale " + std::to_string(p.rescale) +
                                              " is below the Gershgorin bound " + std::to_string(ham->gersh) +
                                              " of H");
        if (!(p.bessel_eps > 0.0))
            p.bessel_eps = 1e-14;
        if (!(feps > 0.0))
            feps = 1e-14;
        std::vector<double> a;
        if (!fermi_coefficients(p.rescale, mu, kT, feps, a))
            return fail(TBPM_ERR_ARG, "the Fermi series did not converge (kT too small for the rescale?)");
        // two coefficients at least: the series kernels start with terms 0 and 1
        MF = std::max<int>((int)a.size(), 2);
        a.resize((size_t)MF, 0.0);
        fa.assign(2 * (size_t)MF, 0.0);
        fb.assign(2 * (size_t)MF, 0.0);
        for (int m = 0; m < MF; ++m) {
            fa[2 * (size_t)m] = a[(size_t)m];
            fb[2 * (size_t)m] = (m == 0 ? 1.0 : 0.0) - a[(size_t)m];
        }
        coeff.assign(2 * 4096, 0.0);
        M = chebyshev_coefficients(3.141592653589793238462643383279, p.bessel_eps, 4096, coeff.data());
        if (M < 2)
            return fail(TBPM_ERR_ARG, "Chebyshev series could not be truncated");
        coeff.resize(2 * (size_t)M);
        elem = ham->dtype == TBPM_C128 ? 16 : 8;
        shape = choose_shape(ham, 1, ctx->num_cu, p.lanes_per_row);
        pairs = ham->patched && pair_supported(ham->ell_w, ham->patch_rows);
        clenshaw = ctx->series.load() == TBPM_SERIES_CLENSHAW;
        max_grid = std::max(shape.grid, op_dot_grid(ham->n));
        if (pairs)
            max_grid = std::max<int64_t>(max_grid, ham->npatch);
        return TBPM_OK;
    }

    size_t footprint() const
    {
        return 8 * (size_t)ham->n * elem + (size_t)max_grid * 4 * sizeof(double) +
               ((size_t)p.num_time_steps + 1) * 3 * sizeof(double);
    }

    void release()
    {
        void *bufs[] = {T0, W, S1, S2, O, Q, X1, X2, partials, corr_dev, norms_dev};
        for (void *b : bufs)
            if (b)
                ctx->dev_free(b);
        T0 = W = S1 = S2 = O = Q = X1 = X2 = nullptr;
        partials = corr_dev = norms_dev = nullptr;
    }

    tbpm_status run(hipStream_t st, double *corr)
    {
        const int64_t n = ham->n;
        const size_t vb = (size_t)n * elem;
        const size_t nt1 = (size_t)p.num_time_steps + 1;
        void **vecs[] = {&T0, &W, &S1, &S2, &O, &Q, &X1, &X2};
        for (void **v : vecs)
            if (!(*v = ctx->dev_alloc(vb)))
                return fail(TBPM_ERR_OOM, "device allocation of the response vectors failed");
        partials = (double *)ctx->dev_alloc((size_t)max_grid * 4 * sizeof(double));
        corr_dev = (double *)ctx->dev_alloc(nt1 * 2 * sizeof(double));
        norms_dev = (double *)ctx->dev_alloc(nt1 * sizeof(double));
        if (!partials || !corr_dev || !norms_dev)
            return fail(TBPM_ERR_OOM, "device allocation of the response buffers failed");
#define RSP_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(TBPM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)
        int nblk = 0;
        std::string err;
        // kernel timing of the time steps (ctx profiling): 4 events per series from the context's pool
        size_t ev_used = 0;
        std::vector<SeriesProfile> profs;
        auto pool = [&](size_t i) -> hipEvent_t {
            while (ctx->events.size() <= i) {
                hipEvent_t e = nullptr;
                if (hipEventCreate(&e) != hipSuccess)
                    return nullptr;
                ctx->events.push_back(e);
            }
            return ctx->events[i];
        };
        auto series = [&](const std::vector<double> &c, int m, void *in, void *out, bool timed) -> tbpm_status {
            SeriesBufs bf{in, Q, out, X1, X2};
            SeriesProfile sp{};
            if (timed) {
                for (int i = 0; i < 4; ++i)
                    if (!(sp.ev[i] = pool(ev_used + i)))
                        return fail(TBPM_ERR_HIP, "event creation failed");
                ev_used += 4;
                if (hipEventRecord(sp.ev[0], st) != hipSuccess)
                    return fail(TBPM_ERR_HIP, "event record failed");
            }
            tbpm_status s = apply_series(ham, st, shape, pairs, clenshaw, c.data(), m, p.rescale, bf, false, nullptr,
                                         partials, &nblk, timed ? &sp : nullptr, err);
            if (timed)
                profs.push_back(sp);
            return s == TBPM_OK ? s : fail(s, err);
        };
        const bool prof = ctx->profiling;
        const int32_t *perm = ham->patched ? ham->old_of_new : nullptr;
        tbpm_status s;
        for (int r = 0; r < p.num_vectors; ++r) {
            RSP_HIP(launch_init_random(ham->dtype, T0, T0, n, 1, p.seed, (int64_t)p.first_vector + r, perm, st));
            RSP_HIP(launch_op_apply(ham->dtype, opb->rp, opb->rp64, opb->col, opb->val, n, T0, W, st));  // B phi
            if ((s = series(fa, MF, T0, S2, false)) != TBPM_OK)          // phi2 = f(H) phi
                return s;
            if ((s = series(fb, MF, W, S1, false)) != TBPM_OK)           // phi1 = (1 - f(H)) B phi
                return s;
            for (size_t k = 0;; ++k) {
                RSP_HIP(launch_op_dot(ham->dtype, opa->rp, opa->rp64, opa->col, opa->val, n, S2, S1, partials, st));
                RSP_HIP(launch_reduce(partials, op_dot_grid(n), 1, corr_dev + 2 * k, norms_dev + k, st));
                if (k + 1 == nt1)
                    break;
                if ((s = series(coeff, M, S1, O, prof)) != TBPM_OK)
                    return s;
                std::swap(S1, O);
                if ((s = series(coeff, M, S2, O, prof)) != TBPM_OK)
                    return s;
                std::swap(S2, O);
            }
            RSP_HIP(hipMemcpyAsync(corr + (size_t)r * nt1 * 2, corr_dev, nt1 * 16, hipMemcpyDeviceToHost, st));
            RSP_HIP(hipStreamSynchronize(st));
            for (const SeriesProfile &sp : profs) {
                for (int kind = 0; kind < 3; ++kind) {
                    float ms = 0.0f;
                    RSP_HIP(hipEventElapsedTime(&ms, sp.ev[kind], sp.ev[kind + 1]));
                    ctx->kernel_ms[kind] += ms;
                    ctx->kernel_launches[kind] += sp.launches[kind];
                }
            }
            profs.clear();
            ev_used = 0;
        }
#undef RSP_HIP
        return TBPM_OK;
    }
};

}  // namespace tbpm

using namespace tbpm;

extern "C" {

tbpm_status tbpm_build_operator(tbpm_ctx *ctx, const tbpm_ham *ref, const tbpm_csr *op, tbpm_ham **out)
{
    if (!ctx)
        return TBPM_ERR_ARG;
    if (!ref || !op || !out || ref->ctx != ctx) {
        ctx->last_error = "ref (of this context), op and out are required";
        return TBPM_ERR_ARG;
    }
    *out = nullptr;
    if (op->n != ref->n) {
        ctx->last_error = "the operator's dimension differs from H's";
        return TBPM_ERR_ARG;
    }
    if (!ref->patched)
        return tbpm_build_csr(ctx, op, ref->dtype, TBPM_FMT_CSR, 0, out);
    if (op->on_device) {
        ctx->last_error = "an operator for a patch-reordered H must be given in host memory";
        return TBPM_ERR_ARG;
    }
    // renumber rows and columns as H was: new row i' = new_of_old[i], columns likewise, sorted per row
    const int64_t n = op->n, nnz = op->nnz;
    if (!op->row_ptr || (nnz > 0 && (!op->col || !op->val)) || op->row_ptr[0] != 0 || op->row_ptr[n] != nnz) {
        ctx->last_error = "malformed operator CSR";
        return TBPM_ERR_CSR;
    }
    const std::vector<int32_t> &no = ref->new_of_old;
    std::vector<int32_t> old_of_new((size_t)n);
    for (int64_t i = 0; i < n; ++i)
        old_of_new[(size_t)no[(size_t)i]] = (int32_t)i;
    std::vector<int64_t> rp((size_t)n + 1, 0);
    std::vector<int32_t> col((size_t)std::max<int64_t>(nnz, 1));
    std::vector<double> val(2 * (size_t)std::max<int64_t>(nnz, 1));
    std::vector<std::pair<int32_t, int64_t>> row;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t o = old_of_new[(size_t)r];
        const int64_t b = op->row_ptr[o], e = op->row_ptr[o + 1];
        if (e < b) {
            ctx->last_error = "malformed operator CSR";
            return TBPM_ERR_CSR;
        }
        row.clear();
        for (int64_t j = b; j < e; ++j) {
            const int32_t c = op->col[j];
            if (c < 0 || c >= n) {
                ctx->last_error = "operator column index out of range";
                return TBPM_ERR_CSR;
            }
            row.emplace_back(no[(size_t)c], j);
        }
        std::sort(row.begin(), row.end());
        const int64_t base = rp[(size_t)r];
        for (size_t q = 0; q < row.size(); ++q) {
            col[(size_t)(base + (int64_t)q)] = row[q].first;
            val[2 * (size_t)(base + (int64_t)q)] = op->val[2 * row[q].second];
            val[2 * (size_t)(base + (int64_t)q) + 1] = op->val[2 * row[q].second + 1];
        }
        rp[(size_t)r + 1] = base + (int64_t)row.size();
    }
    tbpm_csr c2{};
    c2.n = n;
    c2.nnz = nnz;
    c2.row_ptr = rp.data();
    c2.col = col.data();
    c2.val = val.data();
    c2.on_device = 0;
    return tbpm_build_csr(ctx, &c2, ref->dtype, TBPM_FMT_CSR, 0, out);
}

tbpm_status tbpm_response_corr(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_ham *op_a, const tbpm_ham *op_b,
                               const tbpm_params *params, double mu, double kT, double fermi_eps, double *corr)
{
    if (!ctx)
        return TBPM_ERR_ARG;
    if (!ham || !params || !corr || ham->ctx != ctx) {
        ctx->last_error = "ham (of this context), params and corr are required";
        return TBPM_ERR_ARG;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
        ctx->last_error = "hipSetDevice failed";
        return TBPM_ERR_HIP;
    }
    TraceRange range("tbpm_response_corr");
    ResponseRun run{ctx, ham, op_a, op_b, *params, mu, kT, fermi_eps};
    tbpm_status s = run.setup();
    if (s == TBPM_OK)
        s = run.run(ctx->stream, corr);
    if (s != TBPM_OK)
        (void)hipStreamSynchronize(ctx->stream);
    run.release();
    if (s != TBPM_OK)
        ctx->last_error = run.error;
    return s;
}




}  // extern "C"
