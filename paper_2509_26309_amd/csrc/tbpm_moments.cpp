// Chebyshev moments of random-phase vectors (kernel polynomial method).
//
// mu_m = <psi0|T_m(H/rho)|psi0>, m < N, the expansion coefficients behind both
// the DOS and the correlation function: since
// exp(-i x y) = sum_m (2 - delta_m0) (-i)^m J_m(x) T_m(y), the correlation at
// t_k = k pi / rho is C(t_k) = sum_m (2 - delta_m0) (-i)^m J_m(k pi) mu_m.  The
// time-evolution series of TBPLaS 2.0 ("Migration to C++") is that expansion
// at x = pi applied step by step; the moments give every t_k from one
// recurrence.
//
// Doubling: with p_m = T_m(H/rho) psi0 and T_m T_n = (T_{m+n} + T_{|m-n|}) / 2,
//   mu_2m   = 2 <p_m|p_m>   - mu_0,
//   mu_2m+1 = 2 <p_m|p_m+1> - mu_1,
// so N moments take ceil(N/2) products with H.  Launch j forms p_{j+1} from
// p_j (and p_{j-1}, overwritten in place) and sums both inner products of
// row j into per-workgroup partials; the partials of up to `chunk` launches
// are reduced in one fixed-order pass.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "tbpm_engine.h"
#include "tbpm_trace.h"

namespace tbpm {


struct MomentRun {
    tbpm_ctx *ctx;
    const tbpm_ham *ham;
    tbpm_params p;
    int num;                          // moments per vector
    int kmax;                         // products with H per vector
    int bmax = 1;
    size_t elem = 16;
    std::vector<std::pair<int, int>> blocks;
    int max_grid = 8;
    int chunk = 1;
    bool pairs = false;               // fused pairs of products (pair_kernel, moment mode)
    void *va = nullptr, *vb = nullptr, *vc = nullptr, *vd = nullptr;
    std::vector<int64_t> site_rows;   // site-localised states (stored rows), else random phases
    // light cone of site-localised states on a patch-reordered H: p_j is zero
    // beyond j row hops of the block's sites, so product j (forming p_j+1)
    // needs only the patches holding a row within j + 1 hops.  A breadth-first
    // search over H's rows, cut off at the last product, gives each patch the
    // hop distance of its nearest row; order: patches by that distance,
    // level_end[d]: how many are within d.  Patches never reached are skipped.
    bool light_cone = false;
    bool no_cone = false;             // compute every row (for comparisons)
    std::vector<int32_t> order;
    std::vector<int64_t> level_end;
    std::vector<int32_t> row_dist;    // [n], -1 = not reached (reset after each block)
    std::vector<int32_t> visited;
    int32_t *d_order = nullptr;
    double *partials = nullptr, *raw = nullptr, *mu_dev = nullptr;
    std::string error;

    tbpm_status fail(tbpm_status s, const std::string &m)
    {
        error = m;
        return s;
    }

    int64_t within(int64_t d) const
    {
        if (level_end.empty())
            return 0;
        return level_end[(size_t)std::min<int64_t>(d, (int64_t)level_end.size() - 1)];
    }

    tbpm_status fetch_columns()
    {
        std::lock_guard<std::mutex> lock(ham->host_mu);
        if (!ham->h_ell_col.empty())
            return TBPM_OK;
        std::vector<int32_t> c((size_t)ham->ell_w * (size_t)ham->ell_ld);
        if (hipMemcpy(c.data(), ham->col, c.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(TBPM_ERR_HIP, "copy of the stored columns failed");
        ham->h_ell_col.swap(c);
        return TBPM_OK;
    }

    void plan_cone(int r0, int B, int32_t depth)
    {
        const int64_t n = ham->n, ld = ham->ell_ld;
        const int w = ham->ell_w;
        const int32_t *col = ham->h_ell_col.data();
        if (row_dist.empty())
            row_dist.assign((size_t)n, -1);
        visited.clear();
        for (int b = 0; b < B; ++b) {
            const int32_t r = (int32_t)site_rows[(size_t)r0 + b];
            if (row_dist[(size_t)r] < 0) {
                row_dist[(size_t)r] = 0;
                visited.push_back(r);
            }
        }
        for (size_t head = 0; head < visited.size(); ++head) {
            const int32_t r = visited[head];
            const int32_t d = row_dist[(size_t)r];
            if (d >= depth)
                continue;
            for (int s2 = 0; s2 < w; ++s2) {
                const int32_t c = col[(size_t)s2 * (size_t)ld + (size_t)r];
                if (row_dist[(size_t)c] < 0) {
                    row_dist[(size_t)c] = d + 1;
                    visited.push_back(c);
                }
            }
        }
        // patch distance: its nearest row; then patches ordered by distance
        const int64_t np = ham->npatch;
        std::vector<int32_t> pd((size_t)np, -1);
        const std::vector<int32_t> &pp = ham->h_patch_ptr;
        for (int32_t r : visited) {
            const int32_t q = (int32_t)(std::upper_bound(pp.begin(), pp.end(), r) - pp.begin()) - 1;
            const int32_t d = row_dist[(size_t)r];
            if (pd[(size_t)q] < 0 || d < pd[(size_t)q])
                pd[(size_t)q] = d;
            row_dist[(size_t)r] = -1;                 // reset for the next block
        }
        std::vector<int64_t> cnt((size_t)depth + 2, 0);
        for (int64_t q = 0; q < np; ++q)
            if (pd[(size_t)q] >= 0)
                ++cnt[(size_t)pd[(size_t)q]];
        level_end.assign((size_t)depth + 1, 0);
        std::vector<int64_t> pos((size_t)depth + 2, 0);
        int64_t acc = 0;
        for (int32_t d = 0; d <= depth; ++d) {
            pos[(size_t)d] = acc;
            acc += cnt[(size_t)d];
            level_end[(size_t)d] = acc;
        }
        order.assign((size_t)acc, 0);
        for (int64_t q = 0; q < np; ++q)
            if (pd[(size_t)q] >= 0)
                order[(size_t)pos[(size_t)pd[(size_t)q]]++] = (int32_t)q;
    }

    tbpm_status setup()
    {
        if (!(p.rescale > 0.0) || !std::isfinite(p.rescale))
            return fail(TBPM_ERR_ARG, "rescale must be positive");
        if (p.num_vectors < 1)
            return fail(TBPM_ERR_ARG, "num_vectors must be >= 1");
        if (p.block < 0 || p.block > 64)
            return fail(TBPM_ERR_ARG, "block must be in 0..64");
        if (p.first_vector < 0)
            return fail(TBPM_ERR_ARG, "first_vector must be >= 0");
        if (p.num_ldos_sites != 0)
            return fail(TBPM_ERR_ARG, "the moment route takes no LDOS sites");
        if (p.lanes_per_row != 0 && p.lanes_per_row != 1 && p.lanes_per_row != 2 && p.lanes_per_row != 4 &&
            p.lanes_per_row != 8 && p.lanes_per_row != 16)
            return fail(TBPM_ERR_ARG, "lanes_per_row must be 0, 1, 2, 4, 8 or 16");
        if (num < 1)
            return fail(TBPM_ERR_ARG, "num_moments must be >= 1");
        for (int64_t &s : site_rows) {
            if (s < 0 || s >= ham->n)
                return fail(TBPM_ERR_ARG, "site out of range");
            if (ham->patched)
                s = ham->new_of_old[(size_t)s];
        }
        light_cone = !site_rows.empty() && ham->patched && !ham->h_patch_ptr.empty() && !no_cone;
        if (p.rescale < ham->gersh)
            return fail(TBPM_ERR_RESCALE, "rescale " + std::to_string(p.rescale) +
                                              " is below the Gershgorin bound " + std::to_string(ham->gersh) +
                                              " of H");
        kmax = (num + 1) / 2;
        elem = ham->dtype == TBPM_C128 ? 16 : 8;
        blocks = split_blocks(ham, &p, false);     // moment products take single terms on blocks
        bmax = 1;
        for (auto &blk : blocks)
            bmax = std::max(bmax, blk.second);
        for (auto &blk : blocks)
            max_grid = std::max({max_grid, choose_shape(ham, blk.second, ctx->num_cu, p.lanes_per_row).grid,
                                 choose_shape(ham, blk.second, ctx->num_cu, p.lanes_per_row, false).grid});
        // two products with H per pass: patch-reordered H, single-vector blocks
        pairs = false;
        if (ham->patched && pair_supported(ham->ell_w, ham->patch_rows) && kmax >= 3)
            for (auto &blk : blocks)
                pairs = pairs || blk.second == 1;
        if (pairs)
            max_grid = std::max<int64_t>(max_grid, ham->npatch);
        // partials of up to 64 launches, at most about 32 MiB of them
        const size_t per = (size_t)max_grid * bmax * 4 * sizeof(double);
        chunk = (int)std::max<size_t>(pairs ? 2 : 1, std::min<size_t>(64, ((size_t)32 << 20) / per));
        chunk = std::min(chunk, kmax);
        return TBPM_OK;
    }

    size_t footprint() const
    {
        const size_t n = (size_t)ham->n;
        return (pairs ? 4 : 2) * n * (size_t)bmax * elem + (size_t)chunk * max_grid * bmax * 4 * sizeof(double) +
               (size_t)bmax * kmax * 4 * sizeof(double) + (size_t)bmax * num * 2 * sizeof(double);
    }

    void release()
    {
        void *bufs[] = {va, vb, vc, vd, partials, raw, mu_dev, d_order};
        for (void *b : bufs)
            if (b)
                ctx->dev_free(b);
        va = vb = vc = vd = nullptr;
        d_order = nullptr;
        partials = raw = mu_dev = nullptr;
    }

    tbpm_status run(hipStream_t st, double *mu_host)
    {
        const size_t n = (size_t)ham->n;
        va = ctx->dev_alloc(n * bmax * elem);
        vb = ctx->dev_alloc(n * bmax * elem);
        partials = (double *)ctx->dev_alloc((size_t)chunk * max_grid * bmax * 4 * sizeof(double));
        raw = (double *)ctx->dev_alloc((size_t)bmax * kmax * 4 * sizeof(double));
        mu_dev = (double *)ctx->dev_alloc((size_t)bmax * num * 2 * sizeof(double));
        if (pairs) {
            vc = ctx->dev_alloc(n * elem);
            vd = ctx->dev_alloc(n * elem);
        }
        if (light_cone) {
            d_order = (int32_t *)ctx->dev_alloc((size_t)ham->npatch * 4);
            tbpm_status fs = fetch_columns();
            if (fs != TBPM_OK)
                return fs;
        }
        if (!va || !vb || !partials || !raw || !mu_dev || (pairs && (!vc || !vd)) || (light_cone && !d_order))
            return fail(TBPM_ERR_OOM, "device allocation of the moment buffers failed");
        const int fmt = ham->format == TBPM_FMT_CSR ? F_CSR : F_ELL;
        size_t ev_used = 0;
        // kernel timing: span (first event, last event, kind, launches)
        struct Span {
            size_t a, b;
            int kind, launches;
        };
        std::vector<Span> spans;
        const bool prof = ctx->profiling;
        auto record = [&](hipStream_t s2) -> hipError_t {
            while (ctx->events.size() <= ev_used) {
                hipEvent_t ne = nullptr;
                hipError_t e = hipEventCreate(&ne);
                if (e != hipSuccess)
                    return e;
                ctx->events.push_back(ne);
            }
            return hipEventRecord(ctx->events[ev_used++], s2);
        };
#define MOM_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(TBPM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)
        for (auto &blk : blocks) {
            const int r0 = blk.first, B = blk.second;
            // the light cone lists patches: the staged kernel takes every patch
            const KernelShape shape = choose_shape(ham, B, ctx->num_cu, p.lanes_per_row, !light_cone);
            const int64_t stride = (int64_t)shape.grid * B * 4;
            // psi0 itself is p_0; init writes the same state to both of its targets
            if (!site_rows.empty()) {
                SiteRows sr{};
                for (int b = 0; b < B; ++b)
                    sr.r[b] = site_rows[(size_t)r0 + b];
                MOM_HIP(launch_init_sites(ham->dtype, va, va, ham->n, B, sr, st));
                if (light_cone) {
                    // rows never reached stay exact zeros in every buffer
                    // the last product (index kmax - 1, or kmax with a pair) forms rows within kmax + 1 hops
                    plan_cone(r0, B, kmax + 1);
                    MOM_HIP(hipMemcpyAsync(d_order, order.data(), order.size() * 4, hipMemcpyHostToDevice, st));
                    MOM_HIP(hipMemsetAsync(vb, 0, n * B * elem, st));
                    if (pairs && B == 1) {
                        MOM_HIP(hipMemsetAsync(vc, 0, n * elem, st));
                        MOM_HIP(hipMemsetAsync(vd, 0, n * elem, st));
                    }
                }
            } else {
                MOM_HIP(launch_init_random(ham->dtype, va, va, ham->n, B, p.seed, (int64_t)p.first_vector + r0,
                                           ham->patched ? ham->old_of_new : nullptr, st));
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
            if (ham->patched) {
                a.patch_ptr = ham->patch_ptr;
                a.npatch = ham->npatch;
                a.lcol = ham->lcol;
                a.halo_ptr = ham->halo_ptr;
                a.halo_rows = ham->halo_rows;
            }
            void *X = va, *Y = vb;
            // single products j0 .. j0+cnt-1 (timed as `kind`), reduced together
            auto singles = [&](int j0, int cnt, int kind) -> tbpm_status {
                size_t ia = ev_used;
                if (prof)
                    MOM_HIP(record(st));
                for (int j = j0; j < j0 + cnt; ++j) {
                    a.x = X;
                    a.y = Y;
                    a.scale = (j == 0 ? 1.0 : 2.0) / p.rescale;
                    a.partials = partials + (int64_t)(j - j0) * stride;
                    if (light_cone) {
                        a.plist = d_order;
                        a.pcount = within(j + 1);
                        a.patch_ptr = ham->patch_ptr;
                        a.patch_tiles = (ham->patch_rows + rows_per_tile(shape) - 1) / rows_per_tile(shape);
                    }
                    MOM_HIP(launch_term(j == 0 ? K_MOM0 : K_MOM, ham->dtype, fmt, a, shape, st));
                    std::swap(X, Y);
                }
                if (prof) {
                    const size_t ib = ev_used;
                    MOM_HIP(record(st));
                    spans.push_back({ia, ib, kind, cnt});
                }
                MOM_HIP(launch_moment_reduce(partials, shape.grid, B, stride, cnt, j0, raw, kmax, st));
                return TBPM_OK;
            };
            tbpm_status rs = TBPM_OK;
            if (pairs && B == 1) {
                // product 0 alone, then pairs (pair_kernel in moment mode), then a single one if left over
                if ((rs = singles(0, 1, 0)) != TBPM_OK)
                    return rs;
                PairArgs pa{};
                pa.lcol = ham->lcol;
                pa.val = ham->val;
                pa.ld = ham->ell_ld;
                pa.w = ham->ell_w;
                pa.n = ham->n;
                pa.npatch = ham->npatch;
                pa.patch_ptr = ham->patch_ptr;
                pa.halo_ptr = ham->halo_ptr;
                pa.halo_rows = ham->halo_rows;
                pa.hcol = ham->hcol;
                pa.hval = ham->hval;
                pa.vidx = ham->vidx;
                pa.hvidx = ham->hvidx;
                pa.vtab = ham->vtab;
                pa.vdiag = ham->vdiag;
                pa.vdiag_real = ham->vdiag_real;
                pa.ldh = ham->ldh;
                pa.scale = 2.0 / p.rescale;
                const int64_t pstride = ham->npatch * 4;
                void *S1 = vc, *S2 = vd;
                int m = 1;
                while (kmax - m >= 2) {
                    const int npair = std::min(chunk / 2, (kmax - m) / 2);
                    if (light_cone)      // patches left out write no partials
                        MOM_HIP(hipMemsetAsync(partials, 0, (size_t)2 * npair * pstride * sizeof(double), st));
                    const size_t ia = ev_used;
                    if (prof)
                        MOM_HIP(record(st));
                    for (int q = 0; q < npair; ++q) {
                        pa.xin = X;                 // p_m
                        pa.yin = Y;                 // p_m-1
                        pa.yout = S1;               // p_m+1
                        pa.xout = S2;               // p_m+2
                        pa.partials = partials + (int64_t)(2 * q) * pstride;
                        pa.partials2 = partials + (int64_t)(2 * q + 1) * pstride;
                        if (light_cone) {        // forms p_m+1 and p_m+2, m = current product index
                            pa.plist = d_order;
                            pa.pcount = within(m + 2 * q + 2);
                        }
                        MOM_HIP(launch_pair(PAIR_MOM, ham->dtype, pa, ham->patch_rows, st));
                        void *ox = X, *oy = Y;
                        X = S2;
                        Y = S1;
                        S1 = ox;
                        S2 = oy;
                    }
                    if (prof) {
                        const size_t ib = ev_used;
                        MOM_HIP(record(st));
                        spans.push_back({ia, ib, 1, npair});
                    }
                    MOM_HIP(launch_moment_reduce(partials, (int)ham->npatch, 1, pstride, 2 * npair, m, raw, kmax,
                                                 st));
                    m += 2 * npair;
                }
                if (m < kmax && (rs = singles(m, 1, 2)) != TBPM_OK)
                    return rs;
            } else {
                for (int j0 = 0; j0 < kmax; j0 += chunk) {
                    // timed: product 0 alone (kind 0), the others per chunk (kind 1)
                    if (j0 == 0) {
                        if ((rs = singles(0, 1, 0)) != TBPM_OK)
                            return rs;
                        if (std::min(chunk, kmax) > 1 && (rs = singles(1, std::min(chunk, kmax) - 1, 1)) != TBPM_OK)
                            return rs;
                    } else if ((rs = singles(j0, std::min(chunk, kmax - j0), 1)) != TBPM_OK) {
                        return rs;
                    }
                }
            }
            MOM_HIP(launch_moment_finish(raw, kmax, B, num, mu_dev, st));
            MOM_HIP(hipMemcpyAsync(mu_host + (size_t)r0 * num * 2, mu_dev, (size_t)B * num * 16,
                                   hipMemcpyDeviceToHost, st));
            MOM_HIP(hipStreamSynchronize(st));
            for (const Span &sp : spans) {
                float ms = 0.0f;
                MOM_HIP(hipEventElapsedTime(&ms, ctx->events[sp.a], ctx->events[sp.b]));
                ctx->kernel_ms[sp.kind] += ms;
                ctx->kernel_launches[sp.kind] += sp.launches;
            }
            spans.clear();
            ev_used = 0;
        }
#undef MOM_HIP
        return TBPM_OK;
    }
};

}  // namespace tbpm

using namespace tbpm;

extern "C" {

tbpm_status tbpm_moments_footprint(const tbpm_ham *ham, const tbpm_params *params, int32_t num_moments,
                                   size_t *bytes)
{
    if (!ham || !params || !bytes)
        return TBPM_ERR_ARG;
    MomentRun m{ham->ctx, ham, *params, num_moments, 0};
    tbpm_status s = m.setup();
    if (s != TBPM_OK)
        return s;
    *bytes = m.footprint();
    return TBPM_OK;
}

static tbpm_status moments_sync(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params, int32_t num_moments,
                                double *mu, const int64_t *sites, int32_t num_sites);

tbpm_status tbpm_chebyshev_moments(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params,
                                   int32_t num_moments, double *mu)
{
    return moments_sync(ctx, ham, params, num_moments, mu, nullptr, 0);
}

tbpm_status tbpm_site_moments(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params, const int64_t *sites,
                              int32_t num_sites, int32_t num_moments, double *mu)
{
    if (!ctx)
        return TBPM_ERR_ARG;
    if (num_sites < 1 || !sites) {
        ctx->last_error = "at least one site is required";
        return TBPM_ERR_ARG;
    }
    return moments_sync(ctx, ham, params, num_moments, mu, sites, num_sites);
}

static tbpm_status moments_sync(tbpm_ctx *ctx, const tbpm_ham *ham, const tbpm_params *params, int32_t num_moments,
                                double *mu, const int64_t *sites, int32_t num_sites)
{
    if (!ctx)
        return TBPM_ERR_ARG;
    TraceRange range(sites ? "tbpm_site_moments" : "tbpm_chebyshev_moments");
    if (!ham || !params || !mu) {
        ctx->last_error = "ham, params and mu are required";
        return TBPM_ERR_ARG;
    }
    if (ham->ctx != ctx) {
        ctx->last_error = "the Hamiltonian belongs to another context";
        return TBPM_ERR_ARG;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) {
        ctx->last_error = "hipSetDevice failed";
        return TBPM_ERR_HIP;
    }
    MomentRun m{ctx, ham, *params, num_moments, 0};
    if (sites) {
        m.p.num_vectors = num_sites;
        m.p.first_vector = 0;
        m.site_rows.assign(sites, sites + num_sites);
    }
    tbpm_status s = m.setup();
    if (s == TBPM_OK)
        s = m.run(ctx->stream, mu);
    if (s != TBPM_OK)
        (void)hipStreamSynchronize(ctx->stream);
    m.release();
    if (s != TBPM_OK)
        ctx->last_error = m.error;
    return s;
}

}  // extern "C"

