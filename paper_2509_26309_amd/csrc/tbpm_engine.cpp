// Propagation engine (see tbpm_engine.h).
//
// One time step of a block of B vectors (TBPLaS 2.0, "Migration to C++"):
//   term 1:       Q = (1/rho) H P,        O = c_0 P + c_1 Q
//   term m >= 2:  Y = (2/rho) H X - Y,    O = O + c_m Y      (X, Y alternate P, Q)
//   last term:    also the partial sums of <psi0|O> and <O|O>
// then psi(t_{k+1}) = O, and the roles rotate (P, Q, O) <- (O, P, Q).
#include "tbpm_engine.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace tbpm {

#define JOB_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(TBPM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

static hipEvent_t pool_event(tbpm_ctx *ctx, size_t i);

static int pow2_floor(int v)
{
    int p = 1;
    while (p * 2 <= v)
        p *= 2;
    return p;
}

int choose_block(const tbpm_ham *ham, const tbpm_params *p, bool pairs_ok)
{
    if (p->block > 0)
        return std::min(64, pow2_floor(p->block));
    if (ham->tuned_block > 0)
        return std::min(ham->tuned_block, pow2_floor(std::max(1, p->num_vectors)));
    // patch-reordered H: one vector at a time takes the fused pairs, which
    // move fewer bytes per vector and term than any block of complex128
    // vectors (3 vector passes per term against 5, H being small); complex64
    // blocks of 8 and 16 have the staged kernel, and blocks of 8 the fused
    // pairs where H allows them (a block of 16 splits every 128-byte row
    // between two workgroups: 10% slower per vector on the AB bilayer)
    if (ham->patched) {
        if (ham->dtype == TBPM_C128)
            return 1;
        const int b = std::min(16, pow2_floor(std::max(1, p->num_vectors)));
        return (b == 16 && pairs_ok && block_pairs(ham, 8)) ? 8 : b;
    }
    // H is read once per block: wider blocks amortise it; 16 keeps the
    // [n][B] rows at one or two 128-byte lines
    return std::min(16, pow2_floor(std::max(1, p->num_vectors)));
}

bool block_pairs(const tbpm_ham *ham, int B)
{
    return B > 1 && ham->patched && ham->format == TBPM_FMT_PATCH &&
           bpair_supported(ham->dtype, B, ham->ell_w, ham->patch_rows, ham->max_halo);
}

std::vector<std::pair<int, int>> split_blocks(const tbpm_ham *ham, const tbpm_params *p, bool pairs_ok)
{
    const int b0 = choose_block(ham, p, pairs_ok);
    // the library's own choice on patch-reordered H: blocks narrower than 8
    // have no staged kernel, so their vectors go one at a time (fused pairs)
    const bool own = p->block <= 0 && ham->tuned_block <= 0 && ham->patched;
    std::vector<std::pair<int, int>> blocks;
    int r = 0, left = p->num_vectors;
    while (left > 0) {
        int b = std::min(b0, pow2_floor(left));
        if (own && b < 8)
            b = 1;
        blocks.emplace_back(r, b);
        r += b;
        left -= b;
    }
    return blocks;
}

KernelShape choose_shape(const tbpm_ham *ham, int B, int num_cu, int lanes_per_row, bool staged_ok)
{
    KernelShape s{};
    s.B = B;
    if (B > 1)
        s.lr = block_lanes(B, ham->dtype);
    else if (ham->format != TBPM_FMT_CSR)
        s.lr = 1;
    else
        s.lr = lanes_per_row > 0 ? lanes_per_row : ham->lpr;
    s.grid = term_grid(ham->n, s, num_cu);
    if (staged_ok && ham->patched && staged_supported(ham->dtype, B, ham->ell_w, ham->patch_rows)) {
        s.staged = 1;
        s.grid = staged_blocks(B, ham->npatch);
    }
    return s;
}

Job::~Job() { release(); }

tbpm_status Job::fail(tbpm_status s, const std::string &msg)
{
    error = msg;
    return s;
}

tbpm_status Job::setup(tbpm_ctx *c, const tbpm_ham *h, const tbpm_params *prm, hipStream_t stream)
{
    ctx = c;
    ham = h;
    st = stream;
    if (!prm)
        return fail(TBPM_ERR_ARG, "params is NULL");
    p = *prm;
    if (!(p.rescale > 0.0) || !std::isfinite(p.rescale))
        return fail(TBPM_ERR_ARG, "rescale must be positive");
    if (p.num_time_steps < 0)
        return fail(TBPM_ERR_ARG, "num_time_steps must be >= 0");
    if (p.num_vectors < 1)
        return fail(TBPM_ERR_ARG, "num_vectors must be >= 1");
    if (p.block < 0 || p.block > 64)
        return fail(TBPM_ERR_ARG, "block must be in 0..64");
    if (p.first_vector < 0)
        return fail(TBPM_ERR_ARG, "first_vector must be >= 0");
    if (p.num_ldos_sites < 0 || (p.num_ldos_sites > 0 && !p.ldos_sites))
        return fail(TBPM_ERR_ARG, "ldos_sites missing");
    if (p.norm_tol < 0.0)
        return fail(TBPM_ERR_ARG, "norm_tol must be >= 0");
    if (p.lanes_per_row != 0 && p.lanes_per_row != 1 && p.lanes_per_row != 2 && p.lanes_per_row != 4 &&
        p.lanes_per_row != 8 && p.lanes_per_row != 16)
        return fail(TBPM_ERR_ARG, "lanes_per_row must be 0, 1, 2, 4, 8 or 16");
    if (!(p.bessel_eps > 0.0))
        p.bessel_eps = 1e-14;
    if (p.bessel_eps >= 1.0)
        return fail(TBPM_ERR_ARG, "bessel_eps must be < 1");
    if (p.rescale < ham->gersh)
        return fail(TBPM_ERR_RESCALE, "rescale " + std::to_string(p.rescale) + " is below the Gershgorin bound " +
                                          std::to_string(ham->gersh) + " of H");
    if (!site_states.empty()) {
        if ((int64_t)site_states.size() != (int64_t)p.num_vectors)
            return fail(TBPM_ERR_ARG, "one site per vector");
        for (int64_t &s : site_states) {
            if (s < 0 || s >= ham->n)
                return fail(TBPM_ERR_ARG, "site out of range");
            if (ham->patched)
                s = ham->new_of_old[(size_t)s];
        }
    }
    if (!snap_steps.empty() || !qe_energies.empty()) {
        if (p.num_vectors != 1)
            return fail(TBPM_ERR_ARG, "snapshots and quasi-eigenstates take one vector (num_vectors = 1)");
        for (int32_t k2 : snap_steps)
            if (k2 < 0 || k2 > p.num_time_steps)
                return fail(TBPM_ERR_ARG, "snapshot step outside 0..num_time_steps");
        for (double e : qe_energies)
            if (!std::isfinite(e))
                return fail(TBPM_ERR_ARG, "quasi-eigenstate energies must be finite");
    }
    sites.assign(p.ldos_sites, p.ldos_sites + p.num_ldos_sites);
    for (int64_t &s : sites) {
        if (s < 0 || s >= ham->n)
            return fail(TBPM_ERR_ARG, "ldos site out of range");
        if (ham->patched)
            s = ham->new_of_old[(size_t)s];         // stored row of the orbital
    }
    p.ldos_sites = nullptr;

    // dt = pi / rho, so tau = rho dt = pi
    const double tau = 3.141592653589793238462643383279;
    const int max_terms = 4096;
    coeff.assign(2 * (size_t)max_terms, 0.0);
    M = chebyshev_coefficients(tau, p.bessel_eps, max_terms, coeff.data());
    if (M < 2)
        return fail(TBPM_ERR_ARG, "Chebyshev series could not be truncated");
    coeff.resize(2 * (size_t)M);

    elem = ham->dtype == TBPM_C128 ? 16 : 8;
    // the forward recurrence may run blocks in fused pairs; Clenshaw's takes single terms
    blocks = split_blocks(ham, &p, ctx->series.load() != TBPM_SERIES_CLENSHAW);
    bmax = 1;
    for (auto &blk : blocks)
        bmax = std::max(bmax, blk.second);
    max_grid = 8;
    for (auto &blk : blocks)
        max_grid = std::max(max_grid, choose_shape(ham, blk.second, ctx->num_cu, p.lanes_per_row).grid);
    dot_grid = (int)std::min<int64_t>(std::max<int64_t>((ham->n + 255) / 256, 1), 1024);
    max_grid = std::max(max_grid, dot_grid);
    // fused term pairs: patch-reordered H, M - 2 >= 2 recurrence terms, and
    // single-vector blocks or (forward recurrence) complex64 blocks of 8 or 16
    pairs = ham->patched && M >= 4;
    clenshaw = ctx->series.load() == TBPM_SERIES_CLENSHAW;
    bool any_single = false;
    if (pairs) {
        bool any_block = false;
        for (auto &blk : blocks) {
            any_single = any_single || blk.second == 1;
            any_block = any_block || (!clenshaw && block_pairs(ham, blk.second));
        }
        pairs = any_single || any_block;
        max_grid = std::max<int64_t>(max_grid, ham->npatch);
    }
    cross = pairs && any_single && !clenshaw && M >= 6 && M % 2 == 0;
    return TBPM_OK;
}

size_t Job::footprint() const
{
    const size_t n = (size_t)ham->n;
    const size_t nt1 = (size_t)p.num_time_steps + 1;
    size_t b = (cross ? 7 : pairs ? 6 : 4) * n * (size_t)bmax * elem;   // psi0 + three (five, six) rotating vectors
    b += (size_t)max_grid * (size_t)bmax * 4 * sizeof(double);
    b += nt1 * (size_t)bmax * 3 * sizeof(double);          // corr (complex) + norms
    b += sites.size() * (nt1 * 2 * sizeof(double) + sizeof(int64_t));
    if (given_states || final_states || !snap_steps.empty() || !qe_energies.empty())
        b += n * (size_t)bmax * 16;
    b += qe_energies.size() * n * 16;
    return b;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t Job::arena_need() const
{
    const size_t n = (size_t)ham->n;
    const size_t vb_bytes = align256(n * (size_t)bmax * elem);
    const size_t nt1 = (size_t)p.num_time_steps + 1;
    return (cross ? 7 : pairs ? 6 : 4) * vb_bytes + align256((size_t)max_grid * bmax * 4 * sizeof(double)) +
           align256(nt1 * bmax * 2 * sizeof(double)) + align256(nt1 * bmax * sizeof(double)) + align256(256);
}

tbpm_status Job::allocate()
{
    const size_t n = (size_t)ham->n;
    const size_t vb_bytes = n * (size_t)bmax * elem;
    const size_t nt1 = (size_t)p.num_time_steps + 1;
    arena_used = 0;
    // device memory: the context's allocator, or a carve of the caller's arena
    auto take = [&](size_t bytes) -> void * {
        if (!arena)
            return ctx->dev_alloc(bytes);
        const size_t b = align256(bytes);
        if (arena_used + b > arena_bytes)
            return nullptr;
        void *q = arena + arena_used;
        arena_used += b;
        return q;
    };
    if (arena && (!sites.empty() || given_states || final_states || !snap_steps.empty() || !qe_energies.empty() ||
                  !direct_corr))
        return fail(TBPM_ERR_ARG, "the allocation-free mode takes random-phase correlation runs only");
    psi0 = take(vb_bytes);
    va = take(vb_bytes);
    vb = take(vb_bytes);
    vc = take(vb_bytes);
    partials = (double *)take((size_t)max_grid * bmax * 4 * sizeof(double));
    corr_dev = (double *)take(nt1 * bmax * 2 * sizeof(double));
    norms_dev = (double *)take(nt1 * bmax * sizeof(double));
    div_flag = (int32_t *)take(256);
    bool ok = psi0 && va && vb && vc && partials && corr_dev && norms_dev && div_flag;
    if (ok && pairs) {
        vd = take(vb_bytes);
        ve = take(vb_bytes);
        ok = vd && ve;
    }
    if (ok && cross) {
        vf = take(vb_bytes);
        ok = vf != nullptr;
    }
    if (ok && !sites.empty()) {
        site_dev = (double *)ctx->dev_alloc(sites.size() * nt1 * 2 * sizeof(double));
        sites_dev = (int64_t *)ctx->dev_alloc(sites.size() * sizeof(int64_t));
        ok = site_dev && sites_dev;
    }
    if (ok && (given_states || final_states || !snap_steps.empty() || !qe_energies.empty())) {
        states_dev = (double *)ctx->dev_alloc(n * (size_t)bmax * 16);
        ok = states_dev != nullptr;
    }
    if (ok && !qe_energies.empty()) {
        qe_dev = (double *)ctx->dev_alloc(qe_energies.size() * n * 16);
        ok = qe_dev != nullptr;
    }
    if (!ok) {
        release();
        return fail(arena ? TBPM_ERR_TOO_LARGE : TBPM_ERR_OOM,
                    arena ? "the propagation buffers exceed the scratch area"
                          : "device allocation of the propagation buffers failed");
    }
    // graphs: no per-step host work or timing, enough steps to replay (instantiating
    // a graph allocates, so never in the allocation-free mode)
    graph_mode = !arena && ctx->graphs > 0 && st != nullptr && sites.empty() && snap_steps.empty() &&
                 qe_energies.empty() && p.num_time_steps >= 2 * GRAPH_STEPS &&
                 (ctx->graphs == 2 || (int64_t)n * bmax <= ((int64_t)1 << 21));
    rows_closed = 0;
    JOB_HIP(hipMemsetAsync(div_flag, 0, 4, st));
    if (arena) {
        profile = false;
        cur_block = 0;
        block_open = false;
        return TBPM_OK;
    }
    if (graph_mode && !(kstep = (int32_t *)ctx->dev_alloc(256))) {
        release();
        return fail(TBPM_ERR_OOM, "device allocation of the step counter failed");
    }
    const size_t R = (size_t)p.num_vectors;
    if (hipHostMalloc((void **)&corr_all, nt1 * R * 2 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&norms_all, nt1 * R * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&div_host, 256, hipHostMallocDefault) != hipSuccess) {
        release();
        return fail(TBPM_ERR_OOM, "pinned host allocation failed");
    }
    // vectors of blocks that never run (after an early stop) read as zeros
    std::memset(corr_all, 0, nt1 * R * 2 * sizeof(double));
    std::memset(norms_all, 0, nt1 * R * sizeof(double));
    *div_host = 0;
    if (qe_dev)
        JOB_HIP(hipMemsetAsync(qe_dev, 0, qe_energies.size() * n * 16, st));
    if (!sites.empty()) {
        JOB_HIP(hipMemcpyAsync(sites_dev, sites.data(), sites.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
        JOB_HIP(hipMemsetAsync(site_dev, 0, sites.size() * nt1 * 2 * sizeof(double), st));
    }
    cur_block = 0;
    block_open = false;
    return TBPM_OK;
}

void Job::release()
{
    if (!ctx)
        return;
    drop_graphs();
    void *bufs[] = {psi0, va, vb, vc, vd, ve, vf, partials, corr_dev, norms_dev, site_dev, sites_dev, states_dev,
                    qe_dev, kstep, div_flag};
    if (!arena)
        for (void *b : bufs)
            if (b)
                ctx->dev_free(b);
    arena_used = 0;
    psi0 = va = vb = vc = vd = ve = vf = nullptr;
    partials = corr_dev = norms_dev = site_dev = states_dev = qe_dev = nullptr;
    div_flag = nullptr;
    kstep = nullptr;
    sites_dev = nullptr;
    if (corr_all)
        (void)hipHostFree(corr_all);
    if (norms_all)
        (void)hipHostFree(norms_all);
    if (div_host)
        (void)hipHostFree(div_host);
    corr_all = norms_all = nullptr;
    div_host = nullptr;
}

tbpm_status Job::open_block()
{
    const int r0 = blocks[cur_block].first;
    const int B = blocks[cur_block].second;
    const int64_t n = ham->n;
    shape = choose_shape(ham, B, ctx->num_cu, p.lanes_per_row);
    P = va;
    Q = vb;
    O = vc;
    first_done = false;
    if (!site_states.empty()) {
        SiteRows sr{};
        for (int b = 0; b < B; ++b)
            sr.r[b] = site_states[(size_t)r0 + b];
        JOB_HIP(launch_init_sites(ham->dtype, psi0, P, n, B, sr, st));
    } else if (given_states) {
        JOB_HIP(hipMemcpyAsync(states_dev, given_states + (size_t)r0 * n * 2, (size_t)B * n * 16,
                               hipMemcpyHostToDevice, st));
        JOB_HIP(launch_pack_states(ham->dtype, states_dev, psi0, P, n, B, ham->patched ? ham->old_of_new : nullptr,
                                   st));
    } else {
        JOB_HIP(launch_init_random(ham->dtype, psi0, P, n, B, p.seed, (int64_t)p.first_vector + r0,
                                   ham->patched ? ham->old_of_new : nullptr, st));
    }
    // C(t_0) = <psi0|psi0>
    JOB_HIP(launch_dot_partials(ham->dtype, psi0, P, n, B, partials, dot_grid, st));
    JOB_HIP(launch_reduce(partials, dot_grid, B, corr_dev, norms_dev, st, p.norm_tol, div_flag));
    if (!sites.empty())
        JOB_HIP(launch_ldos_gather(ham->dtype, psi0, P, n, B, sites_dev, (int)sites.size(), site_dev,
                                   p.num_time_steps + 1, 0, st));
    if (graph_mode)
        JOB_HIP(launch_set_counter(kstep, 1, st));
    k = 0;
    block_open = true;
    return emit_outputs();
}

void Job::drop_graphs()
{
    for (StepGraph &g : graphs)
        if (g.exec)
            (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
    graph_B = 0;
}

int Job::find_graph() const
{
    if (graph_B != shape.B)
        return -1;
    for (size_t i = 0; i < graphs.size(); ++i)
        if (graphs[i].sP == P && graphs[i].sQ == Q && graphs[i].sO == O)
            return (int)i;
    return -1;
}

tbpm_status Job::graph_steps()
{
    int gi = find_graph();
    if (gi < 0) {
        if (graph_B != shape.B)
            drop_graphs();
        if ((int)graphs.size() >= MAX_GRAPHS)
            return fail(TBPM_ERR_ARG, "internal: no graph for the current buffer roles");
        // capture: the steps advance k and rotate the buffer roles; the work
        // itself runs when the graph is launched below
        StepGraph sg;
        sg.sP = P;
        sg.sQ = Q;
        sg.sO = O;
        JOB_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        tbpm_status s = TBPM_OK;
        capturing = true;
        graph_terms = 0;
        for (int i = 0; i < GRAPH_STEPS && s == TBPM_OK; ++i)
            s = step();
        capturing = false;
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (s != TBPM_OK) {
            if (g)
                (void)hipGraphDestroy(g);
            return s;
        }
        JOB_HIP(e);
        const hipError_t ei = hipGraphInstantiate(&sg.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        JOB_HIP(ei);
        sg.eP = P;
        sg.eQ = Q;
        sg.eO = O;
        sg.terms = graph_terms;
        graph_B = shape.B;
        graphs.push_back(sg);
        gi = (int)graphs.size() - 1;
    } else {
        // a replay starts from the captured roles and leaves the captured end roles
        k += GRAPH_STEPS;
        P = graphs[gi].eP;
        Q = graphs[gi].eQ;
        O = graphs[gi].eO;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (profile) {
        if (!(e0 = pool_event(ctx, ev_used)) || !(e1 = pool_event(ctx, ev_used + 1)))
            return fail(TBPM_ERR_HIP, "event creation failed");
        graph_ev.push_back(ev_used);
        ev_used += 2;
        JOB_HIP(hipEventRecord(e0, st));
    }
    JOB_HIP(hipGraphLaunch(graphs[gi].exec, st));
    if (profile) {
        JOB_HIP(hipEventRecord(e1, st));
        prof_launch[K_MID] += graphs[gi].terms;
    }
    ctx->graph_replays += 1;
    return TBPM_OK;
}

tbpm_status Job::emit_outputs()
{
    const int64_t n = ham->n;
    const int32_t *perm = ham->patched ? ham->old_of_new : nullptr;
    for (size_t s = 0; s < snap_steps.size(); ++s) {
        if (snap_steps[s] != k)
            continue;
        JOB_HIP(launch_unpack_state(ham->dtype, P, states_dev, n, 1, 0, perm, st));
        JOB_HIP(hipMemcpyAsync(snaps + s * (size_t)n * 2, states_dev, (size_t)n * 16, hipMemcpyDeviceToHost, st));
    }
    if (!qe_energies.empty()) {
        // w_k e^{i E_j t_k}, t_k = k pi / rho, Hann weight (1 without time steps)
        const double pi = 3.141592653589793238462643383279;
        const int nt = p.num_time_steps;
        const double w = nt > 0 ? 0.5 * (1.0 + std::cos(pi * k / nt)) : 1.0;
        const double t = k * pi / p.rescale;
        for (size_t j0 = 0; j0 < qe_energies.size(); j0 += QE_MAX) {
            const int cnt = (int)std::min<size_t>(QE_MAX, qe_energies.size() - j0);
            QeFactors f{};
            for (int j = 0; j < cnt; ++j) {
                const double ph = qe_energies[j0 + j] * t;
                f.re[j] = w * std::cos(ph);
                f.im[j] = w * std::sin(ph);
            }
            JOB_HIP(launch_qe_accumulate(ham->dtype, P, n, qe_dev + j0 * (size_t)n * 2, cnt, f, st));
        }
    }
    return TBPM_OK;
}

static hipEvent_t pool_event(tbpm_ctx *ctx, size_t i)
{
    while (ctx->events.size() <= i) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        ctx->events.push_back(e);
    }
    return ctx->events[i];
}

tbpm_status Job::collect_profile()
{
    if (!profile)
        return TBPM_OK;
    for (size_t i : step_ev) {
        for (int kind = 0; kind < 3; ++kind) {
            float ms = 0.0f;
            JOB_HIP(hipEventElapsedTime(&ms, ctx->events[i + kind], ctx->events[i + kind + 1]));
            ctx->kernel_ms[kind] += ms;
        }
    }
    // a replayed graph is timed as a whole and counted as middle-term time over
    // all of its term launches (its reductions included)
    for (size_t i : graph_ev) {
        float ms = 0.0f;
        JOB_HIP(hipEventElapsedTime(&ms, ctx->events[i], ctx->events[i + 1]));
        ctx->kernel_ms[K_MID] += ms;
    }
    for (int kind = 0; kind < 3; ++kind)
        ctx->kernel_launches[kind] += prof_launch[kind];
    step_ev.clear();
    graph_ev.clear();
    ev_used = 0;
    prof_launch[0] = prof_launch[1] = prof_launch[2] = 0;
    return TBPM_OK;
}

// O = sum_{m<M} c_m T_m(H/rho) P (see tbpm_engine.h).
tbpm_status apply_series(const tbpm_ham *ham, hipStream_t st, const KernelShape &shape, bool pairs, bool clenshaw,
                         const double *c, int M, double rescale, const SeriesBufs &bf, bool dots, const void *psi0,
                         double *partials, int *nblk, SeriesProfile *prof, std::string &err, bool skip_first)
{
#define SER_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            err = std::string(#expr) + ": " + hipGetErrorString(e_);                         \
            return TBPM_ERR_HIP;                                                             \
        }                                                                                    \
    } while (0)
    if (M < 2) {
        err = "a series needs at least two terms";
        return TBPM_ERR_ARG;
    }
    const int B = shape.B;
    const int64_t n = ham->n;
    const int kind_last = dots ? K_LAST : K_MID;
    TermArgs a{};
    a.n = n;
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
    a.psi0 = psi0;
    a.partials = partials;
    if (ham->patched) {
        a.patch_ptr = ham->patch_ptr;
        a.npatch = ham->npatch;
        a.lcol = ham->lcol;
        a.halo_ptr = ham->halo_ptr;
        a.halo_rows = ham->halo_rows;
    }
    const int fmt = ham->format == TBPM_FMT_CSR ? F_CSR : F_ELL;

    if (clenshaw && pairs && B == 1 && M >= 6) {
        // Clenshaw's backward recurrence in fused pairs on patch-reordered H:
        // b_m = c_m P + (2/rho) H b_m+1 - b_m+2 (b_M = b_M+1 = 0), O = c_0 P +
        // (1/rho) H b_1 - b_2.  P stays intact; each pair reads b_m+1, b_m+2
        // and P and writes b_m, b_m-1, so no accumulator is read and written
        // per pair.  Launches: the first pair (b_M-2, b_M-3 from P alone),
        // a single product when M - 5 is odd, (M - 5) / 2 middle pairs, and
        // the last pair (b_1 on chip, O and its correlation partials).  The
        // single product is timed with the first pair, so the middle-term
        // timings cover pairs only.
        PairArgs pa{};
        pa.lcol = ham->lcol;
        pa.val = ham->val;
        pa.ld = ham->ell_ld;
        pa.w = ham->ell_w;
        pa.n = n;
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
        pa.psi = bf.P;
        pa.psi0 = psi0;
        pa.partials = partials;
        pa.scale = 2.0 / rescale;
        pa.scale_b = 2.0 / rescale;
        pa.ka_re = 1.0;
        pa.ka_im = 0.0;
        auto coef = [&](int m, double &re, double &im) {
            re = c[2 * m];
            im = c[2 * m + 1];
        };
        const int mids = (M - 5) / 2;
        const bool single = (M - 5) % 2 == 1;
        // two pairs of b buffers; a pair launch writes (b_m, b_m-1) to (.y, .x) of
        // the pair its inputs are not in, and the last one writes O to .x of the
        // pair left after the middle pairs, which must be bf.O
        void *pr[2][2];                              // [pair][0 = y, 1 = x]
        const int fin = 1 - mids % 2;
        pr[fin][1] = bf.O;
        pr[fin][0] = bf.S1;
        pr[1 - fin][0] = bf.Q;
        pr[1 - fin][1] = bf.S2;
        // first pair: b_M-2 = c_M-1 (2/rho) H P + c_M-2 P; b_M-3 = (2/rho) H b_M-2 - c_M-1 P + c_M-3 P
        pa.xin = bf.P;
        pa.yin = bf.P;                               // not read
        pa.yout = pr[0][0];
        pa.xout = pr[0][1];
        coef(M - 1, pa.ka_re, pa.ka_im);
        coef(M - 2, pa.c0_re, pa.c0_im);
        coef(M - 3, pa.c1_re, pa.c1_im);
        SER_HIP(launch_pair(PAIR_CL_FIRST, ham->dtype, pa, ham->patch_rows, st));
        pa.ka_re = 1.0;
        pa.ka_im = 0.0;
        int cur = 0;                                 // pair holding the two newest b
        void *newest = pr[0][1], *second = pr[0][0];
        int m = M - 4;                               // next b to form
        if (single) {                                // b_m in place of b_m+2
            pa.xin = newest;
            pa.yin = second;
            pa.yout = second;
            coef(m, pa.c0_re, pa.c0_im);
            SER_HIP(launch_pair(PAIR_CL_SINGLE, ham->dtype, pa, ham->patch_rows, st));
            std::swap(newest, second);
            m -= 1;
        }
        if (prof) {
            if (prof->ev[1])
                SER_HIP(hipEventRecord(prof->ev[1], st));
            prof->launches[K_FIRST] += single ? 2 : 1;
        }
        for (int k = 0; k < mids; ++k) {
            pa.xin = newest;
            pa.yin = second;
            pa.yout = pr[1 - cur][0];
            pa.xout = pr[1 - cur][1];
            coef(m, pa.c0_re, pa.c0_im);
            coef(m - 1, pa.c1_re, pa.c1_im);
            SER_HIP(launch_pair(PAIR_CL, ham->dtype, pa, ham->patch_rows, st));
            if (prof)
                prof->launches[K_MID] += 1;
            cur = 1 - cur;
            newest = pr[cur][1];
            second = pr[cur][0];
            m -= 2;
        }
        if (m != 1 || cur != 1 - fin) {
            err = "Clenshaw schedule does not end at b_1";
            return TBPM_ERR_ARG;
        }
        // last pair: b_1 = c_1 P + (2/rho) H b_2 - b_3 (on chip); O = c_0 P + (1/rho) H b_1 - b_2
        if (prof && prof->ev[2])
            SER_HIP(hipEventRecord(prof->ev[2], st));
        pa.xin = newest;
        pa.yin = second;
        pa.yout = pr[fin][0];                        // written only without dots
        pa.xout = pr[fin][1];
        pa.scale_b = 1.0 / rescale;
        coef(1, pa.c0_re, pa.c0_im);
        coef(0, pa.c1_re, pa.c1_im);
        SER_HIP(launch_pair(dots ? PAIR_CL_LAST : PAIR_CL, ham->dtype, pa, ham->patch_rows, st));
        if (prof) {
            prof->launches[K_LAST] += 1;             // by position, as its time
            if (prof->ev[3])
                SER_HIP(hipEventRecord(prof->ev[3], st));
        }
        *nblk = (int)ham->npatch;
        return TBPM_OK;
    }

    if (clenshaw && !(pairs && B == 1 && M >= 4) && M >= 5) {
        // Clenshaw's backward recurrence, one product per launch, in place:
        // b_M-2 = c_M-1 (2/rho) H P + c_M-2 P; b_M-3 = (2/rho) H b_M-2 +
        // (c_M-3 - c_M-1) P (b_M-1 = c_M-1 P folded in); b_m = c_m P +
        // (2/rho) H b_m+1 - b_m+2; O = c_0 P + (1/rho) H b_1 - b_2 in place of
        // b_2.  P stays intact; a middle launch reads b_m+1, b_m+2 and P and
        // writes b_m (4 vector passes against the forward term's 5).  b_m is
        // in A when M - 2 - m is even, so O lands in bf.O.
        void *A = (M % 2 == 0) ? bf.O : bf.Q;
        void *Bv = (M % 2 == 0) ? bf.Q : bf.O;
        a.cl = 1;
        a.psi = bf.P;
        a.scale = 2.0 / rescale;
        a.x = bf.P;
        a.y = A;
        a.ca_re = c[2 * (M - 1)];
        a.ca_im = c[2 * (M - 1) + 1];
        a.cb_re = c[2 * (M - 2)];
        a.cb_im = c[2 * (M - 2) + 1];
        SER_HIP(launch_term(K_FIRST, ham->dtype, fmt, a, shape, st));
        a.x = A;
        a.y = Bv;
        a.no_y = 1;
        a.ca_re = c[2 * (M - 3)] - c[2 * (M - 1)];
        a.ca_im = c[2 * (M - 3) + 1] - c[2 * (M - 1) + 1];
        SER_HIP(launch_term(K_MID, ham->dtype, fmt, a, shape, st));
        a.no_y = 0;
        if (prof) {
            if (prof->ev[1])
                SER_HIP(hipEventRecord(prof->ev[1], st));
            prof->launches[K_FIRST] += 2;
        }
        void *newest = Bv, *second = A;              // b_M-3, b_M-2
        for (int m = M - 4; m >= 0; --m) {
            const bool last = m == 0;
            if (last) {                              // O = c_0 P + (1/rho) H b_1 - b_2
                a.scale = 1.0 / rescale;
                if (prof && prof->ev[2])
                    SER_HIP(hipEventRecord(prof->ev[2], st));
            }
            a.x = newest;
            a.y = second;
            a.ca_re = c[2 * m];
            a.ca_im = c[2 * m + 1];
            SER_HIP(launch_term(last ? kind_last : K_MID, ham->dtype, fmt, a, shape, st));
            if (prof)
                prof->launches[last ? K_LAST : K_MID] += 1;   // by position, as its time
            std::swap(newest, second);
        }
        if (newest != bf.O) {
            err = "Clenshaw schedule does not end in the output buffer";
            return TBPM_ERR_ARG;
        }
        if (prof && prof->ev[3])
            SER_HIP(hipEventRecord(prof->ev[3], st));
        *nblk = shape.grid;
        return TBPM_OK;
    }

    // term 1: Q = (1/rho) H P; O = c0 P + c1 Q (unless a previous launch formed them)
    a.x = bf.P;
    a.y = bf.Q;
    a.out = bf.O;
    if (!skip_first) {
        a.scale = 1.0 / rescale;
        a.ca_re = c[0];
        a.ca_im = c[1];
        a.cb_re = c[2];
        a.cb_im = c[3];
        SER_HIP(launch_term(K_FIRST, ham->dtype, fmt, a, shape, st));
        if (prof)
            prof->launches[K_FIRST] += 1;
    }
    if (prof && prof->ev[1])
        SER_HIP(hipEventRecord(prof->ev[1], st));
    a.scale = 2.0 / rescale;
    *nblk = shape.grid;
    if (pairs && (B == 1 || (!clenshaw && block_pairs(ham, B))) && M >= 4) {
        // terms m = 2..M-1 two at a time (one single term first when their number is odd)
        void *cx = bf.Q, *cy = bf.P, *sp1 = bf.S1, *sp2 = bf.S2;
        int m = 2;
        if ((M - 2) % 2 == 1) {
            a.x = cx;
            a.y = cy;
            a.ca_re = c[2 * m];
            a.ca_im = c[2 * m + 1];
            SER_HIP(launch_term(K_MID, ham->dtype, fmt, a, shape, st));
            if (prof)
                prof->launches[K_MID] += 1;
            std::swap(cx, cy);
            ++m;
        }
        PairArgs pa{};
        pa.lcol = ham->lcol;
        pa.val = ham->val;
        pa.ld = ham->ell_ld;
        pa.w = ham->ell_w;
        pa.n = n;
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
        pa.out = bf.O;
        pa.psi0 = psi0;
        pa.scale = 2.0 / rescale;
        pa.scale_b = 2.0 / rescale;
        pa.partials = partials;
        pa.B = B;
        pa.max_halo = ham->max_halo;
        while (m < M) {                                 // an even number of terms remains
            const bool last = (m + 2 == M);
            if (prof && last && prof->ev[2])
                SER_HIP(hipEventRecord(prof->ev[2], st));
            pa.xin = cx;
            pa.yin = cy;
            pa.yout = sp1;
            pa.xout = sp2;
            pa.c0_re = c[2 * m];
            pa.c0_im = c[2 * m + 1];
            pa.c1_re = c[2 * m + 2];
            pa.c1_im = c[2 * m + 3];
            SER_HIP(launch_pair((last && dots) ? PAIR_LAST : PAIR_MID, ham->dtype, pa, ham->patch_rows, st));
            if (prof)
                prof->launches[last ? K_LAST : K_MID] += 1;
            void *ocx = cx, *ocy = cy;
            cx = sp2;
            cy = sp1;
            sp1 = ocx;
            sp2 = ocy;
            m += 2;
        }
        if (prof && prof->ev[3])
            SER_HIP(hipEventRecord(prof->ev[3], st));
        *nblk = (int)ham->npatch;
        return TBPM_OK;
    }
    // terms m = 2..M-1: Y = (2/rho) H X - Y; O += c_m Y
    void *X = bf.Q, *Y = bf.P;
    for (int m = 2; m < M; ++m) {
        a.x = X;
        a.y = Y;
        a.ca_re = c[2 * m];
        a.ca_im = c[2 * m + 1];
        const bool last = (m == M - 1);
        if (prof && last && prof->ev[2])
            SER_HIP(hipEventRecord(prof->ev[2], st));
        SER_HIP(launch_term(last ? kind_last : K_MID, ham->dtype, fmt, a, shape, st));
        if (prof)
            prof->launches[last ? K_LAST : K_MID] += 1;
        std::swap(X, Y);
    }
    if (prof) {
        if (M < 3 && prof->ev[2])
            SER_HIP(hipEventRecord(prof->ev[2], st));
        if (prof->ev[3])
            SER_HIP(hipEventRecord(prof->ev[3], st));
    }
    if (M == 2 && dots)   // no recurrence term: correlation sums from O directly
        *nblk = -1;
    return TBPM_OK;
#undef SER_HIP
}

tbpm_status apply_series_cross(const tbpm_ham *ham, hipStream_t st, const double *c, int M, double rescale,
                               void *P, void *Q, void *O, void *const spare[3], void *keep, const void *psi0,
                               double *partials, SeriesProfile *prof, void **Pn, void **Qn, void **On,
                               std::string &err)
{
#define SER_HIP(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            err = std::string(#expr) + ": " + hipGetErrorString(e_);                         \
            return TBPM_ERR_HIP;                                                             \
        }                                                                                    \
    } while (0)
    if (M < 6 || M % 2 != 0 || !ham->patched) {
        err = "cross-step pairs need patch-reordered H and an even series of at least 6 terms";
        return TBPM_ERR_ARG;
    }
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
    pa.psi0 = psi0;
    pa.partials = partials;
    auto coef = [&](int m, double &re, double &im) {
        re = c[2 * m];
        im = c[2 * m + 1];
    };
    // terms 1 and 2: p_1 = (1/rho) H P to Q, p_2 = (2/rho) H p_1 - P to spare[0],
    // O = c_0 P + c_1 p_1 + c_2 p_2
    pa.xin = P;
    pa.yin = P;                                      // not read
    pa.yout = Q;
    pa.xout = spare[0];
    pa.out = O;
    pa.scale = 1.0 / rescale;
    pa.scale_b = 2.0 / rescale;
    coef(0, pa.c0_re, pa.c0_im);
    coef(1, pa.c1_re, pa.c1_im);
    coef(2, pa.c2_re, pa.c2_im);
    SER_HIP(launch_pair(PAIR_FIRST, ham->dtype, pa, ham->patch_rows, st));
    if (prof) {
        if (prof->ev[1])
            SER_HIP(hipEventRecord(prof->ev[1], st));
        prof->launches[K_FIRST] += 1;
    }
    // terms 3..M-2 in pairs
    void *cx = spare[0], *cy = Q, *sp1 = P, *sp2 = spare[1];
    pa.scale = 2.0 / rescale;
    pa.scale_b = 2.0 / rescale;
    for (int m = 3; m + 1 <= M - 2; m += 2) {
        pa.xin = cx;
        pa.yin = cy;
        pa.yout = sp1;
        pa.xout = sp2;
        coef(m, pa.c0_re, pa.c0_im);
        coef(m + 1, pa.c1_re, pa.c1_im);
        SER_HIP(launch_pair(PAIR_MID, ham->dtype, pa, ham->patch_rows, st));
        if (prof)
            prof->launches[K_MID] += 1;
        void *ocx = cx, *ocy = cy;
        cx = sp2;
        cy = sp1;
        sp1 = ocx;
        sp2 = ocy;
    }
    // term M-1 (x_{M-2} in cx, y_{M-3} in cy) and the next step's term 1, into
    // three vectors none of this launch reads
    void *fr[3] = {sp1, sp2, spare[2]};
    int ko = 0;
    for (int i = 0; i < 3; ++i)
        if (fr[i] == keep)
            ko = i;
    *On = fr[ko];
    *Pn = fr[(ko + 1) % 3];
    *Qn = fr[(ko + 2) % 3];
    pa.xin = cx;
    pa.yin = cy;
    pa.out = O;
    pa.yout = *Pn;
    pa.xout = *Qn;
    pa.out2 = *On;
    pa.scale = 2.0 / rescale;
    pa.scale_b = 1.0 / rescale;
    coef(M - 1, pa.c0_re, pa.c0_im);
    coef(0, pa.c1_re, pa.c1_im);
    coef(1, pa.c2_re, pa.c2_im);
    if (prof && prof->ev[2])
        SER_HIP(hipEventRecord(prof->ev[2], st));
    SER_HIP(launch_pair(PAIR_CROSS, ham->dtype, pa, ham->patch_rows, st));
    if (prof) {
        prof->launches[K_LAST] += 1;
        if (prof->ev[3])
            SER_HIP(hipEventRecord(prof->ev[3], st));
    }
    return TBPM_OK;
#undef SER_HIP
}

void Job::spare_buffers(void *out[3]) const
{
    void *all[6] = {va, vb, vc, vd, ve, vf};
    int j = 0;
    for (void *b : all)
        if (b && b != P && b != Q && b != O && j < 3)
            out[j++] = b;
    for (; j < 3; ++j)
        out[j] = nullptr;
}

void Job::set_roles(void *psi)
{
    void *all[6] = {va, vb, vc, vd, ve, vf};
    P = psi;
    Q = O = nullptr;
    for (void *b : all) {
        if (!b || b == psi)
            continue;
        if (!Q)
            Q = b;
        else if (!O)
            O = b;
    }
}

tbpm_status Job::step()
{
    SeriesProfile sp{};
    if (profile && !capturing) {
        for (int i = 0; i < 4; ++i)
            if (!(sp.ev[i] = pool_event(ctx, ev_used + i)))
                return fail(TBPM_ERR_HIP, "event creation failed");
        step_ev.push_back(ev_used);
        ev_used += 4;
        JOB_HIP(hipEventRecord(sp.ev[0], st));
    }
    const int B = shape.B;
    const int64_t n = ham->n;
    int nblk = shape.grid;
    std::string err;
    SeriesProfile *prof = (profile || capturing) ? &sp : nullptr;
    // the step either straddles into its successor (cross), completes one whose
    // term 1 was applied by the previous step (first_done), or stands alone
    const bool xs = cross && B == 1 && !first_done && k + 1 < p.num_time_steps;
    void *psi_next = O;              // where psi(t_{k+1}) is after the launches
    void *Pn = nullptr, *Qn = nullptr, *On = nullptr;
    tbpm_status s;
    if (xs) {
        void *spare[3];
        spare_buffers(spare);
        s = apply_series_cross(ham, st, coeff.data(), M, p.rescale, P, Q, O, spare, P, psi0, partials, prof, &Pn,
                               &Qn, &On, err);
        psi_next = Pn;
        nblk = (int)ham->npatch;
    } else {
        void *s1 = vd, *s2 = ve;
        if (cross) {
            void *spare[3];
            spare_buffers(spare);
            s1 = spare[0];
            s2 = spare[1];
        }
        SeriesBufs bf{P, Q, O, s1, s2};
        s = apply_series(ham, st, shape, pairs, clenshaw, coeff.data(), M, p.rescale, bf, true, psi0, partials,
                         &nblk, prof, err, cross && first_done);
    }
    if (s != TBPM_OK)
        return fail(s, err);
    for (int kk = 0; kk < 3; ++kk) {
        if (capturing)
            graph_terms += sp.launches[kk];
        else
            prof_launch[kk] += sp.launches[kk];
    }
    if (nblk < 0) {   // no recurrence term: correlation sums from O directly
        JOB_HIP(launch_dot_partials(ham->dtype, psi0, O, n, B, partials, dot_grid, st));
        nblk = dot_grid;
    }
    ++k;
    if (graph_mode)
        JOB_HIP(launch_reduce_step(partials, nblk, B, corr_dev, norms_dev, kstep, st, p.norm_tol, div_flag));
    else
        JOB_HIP(launch_reduce(partials, nblk, B, corr_dev + (size_t)k * B * 2, norms_dev + (size_t)k * B, st,
                              p.norm_tol, div_flag));
    if (!sites.empty())
        JOB_HIP(launch_ldos_gather(ham->dtype, psi0, psi_next, n, B, sites_dev, (int)sites.size(), site_dev,
                                   p.num_time_steps + 1, k, st));
    if (xs) {
        // psi(t_k) in Pn; the next step's p_1 and partial series in Qn, On
        P = Pn;
        Q = Qn;
        O = On;
        first_done = true;
    } else if (cross) {
        first_done = false;
        set_roles(psi_next);
    } else {
        // psi(t_k) now lives in O; the rest are scratch
        void *oldP = P, *oldQ = Q;
        P = O;
        Q = oldP;
        O = oldQ;
    }
    return emit_outputs();
}

tbpm_status Job::close_block()
{
    const int r0 = blocks[cur_block].first;
    const int B = blocks[cur_block].second;
    const size_t R = (size_t)p.num_vectors;
    const size_t nt1 = (size_t)p.num_time_steps + 1;
    if (direct_corr) {
        // allocation-free mode: column b of [N_t+1][B] to the caller's row r0 + b
        for (int b = 0; b < B; ++b) {
            JOB_HIP(hipMemcpy2DAsync(direct_corr + (size_t)(r0 + b) * nt1 * 2, 16, corr_dev + (size_t)b * 2,
                                     (size_t)B * 16, 16, nt1, hipMemcpyDeviceToHost, st));
            if (direct_norms)
                JOB_HIP(hipMemcpy2DAsync(direct_norms + (size_t)(r0 + b) * nt1, 8, norms_dev + b, (size_t)B * 8, 8,
                                         nt1, hipMemcpyDeviceToHost, st));
        }
    } else {
        // columns r0..r0+B-1 of the [N_t+1][R] host arrays
        JOB_HIP(hipMemcpy2DAsync(corr_all + (size_t)r0 * 2, R * 16, corr_dev, (size_t)B * 16, (size_t)B * 16, nt1,
                                 hipMemcpyDeviceToHost, st));
        JOB_HIP(hipMemcpy2DAsync(norms_all + r0, R * 8, norms_dev, (size_t)B * 8, (size_t)B * 8, nt1,
                                 hipMemcpyDeviceToHost, st));
    }
    if (final_states) {
        const int64_t n = ham->n;
        for (int b = 0; b < B; ++b)
            JOB_HIP(launch_unpack_state(ham->dtype, P, states_dev + (size_t)b * n * 2, n, B, b,
                                        ham->patched ? ham->old_of_new : nullptr, st));
        JOB_HIP(hipMemcpyAsync(final_states + (size_t)r0 * n * 2, states_dev, (size_t)B * n * 16,
                               hipMemcpyDeviceToHost, st));
    }
    if (qe_dev) {
        const int64_t n = ham->n;
        for (size_t j = 0; j < qe_energies.size(); ++j) {
            // FP64 accumulators back to the original row order
            JOB_HIP(launch_unpack_state(TBPM_C128, qe_dev + j * (size_t)n * 2, states_dev, n, 1, 0,
                                        ham->patched ? ham->old_of_new : nullptr, st));
            JOB_HIP(hipMemcpyAsync(qe_host + j * (size_t)n * 2, states_dev, (size_t)n * 16, hipMemcpyDeviceToHost,
                                   st));
        }
    }
    block_open = false;
    ++cur_block;
    rows_closed = r0 + B;
    return TBPM_OK;
}

tbpm_status Job::queue_flag_read()
{
    if (p.norm_tol > 0.0 && div_host)
        JOB_HIP(hipMemcpyAsync(div_host, div_flag, 4, hipMemcpyDeviceToHost, st));
    return TBPM_OK;
}

tbpm_status Job::advance(int max_steps)
{
    int done = 0;
    while (cur_block < blocks.size()) {
        if (!block_open) {
            tbpm_status s = open_block();
            if (s != TBPM_OK)
                return s;
        }
        while (k < p.num_time_steps && done < max_steps) {
            // a replay reads and writes the buffers in the roles they had at capture;
            // eager steps (chunk ends) rotate the roles, so replay only a graph
            // captured from the current roles, or capture one while there is room
            const bool roles = !first_done && (graph_B != shape.B || (int)graphs.size() < MAX_GRAPHS ||
                                               find_graph() >= 0);
            if (graph_mode && roles && p.num_time_steps - k >= GRAPH_STEPS && max_steps - done >= GRAPH_STEPS) {
                tbpm_status s = graph_steps();
                if (s != TBPM_OK)
                    return s;
                done += GRAPH_STEPS;
                continue;
            }
            tbpm_status s = step();
            if (s != TBPM_OK)
                return s;
            ++done;
        }
        if (k < p.num_time_steps)
            return TBPM_PENDING;
        tbpm_status s = close_block();
        if (s != TBPM_OK)
            return s;
        if (done >= max_steps && cur_block < blocks.size())
            return TBPM_PENDING;
    }
    return TBPM_OK;
}


tbpm_status Job::finish(double *corr, double *norms, double *ldos, double *corr_mean)
{
    const size_t R = (size_t)p.num_vectors;
    const size_t nt1 = (size_t)p.num_time_steps + 1;
    if (direct_corr) {
        // allocation-free mode: the rows are already in the caller's arrays
        if (corr_mean)
            sample_mean(direct_corr, R, nt1, true, corr_mean);
        if (p.norm_tol > 0.0 && direct_norms) {
            for (size_t i = 0; i < R * nt1; ++i)
                if (!(std::fabs(direct_norms[i] - 1.0) <= p.norm_tol))
                    return fail(TBPM_ERR_DIVERGED, "norm of vector " + std::to_string(i / nt1) + " at step " +
                                                       std::to_string(i % nt1) + " is " +
                                                       std::to_string(direct_norms[i]) + " (tolerance " +
                                                       std::to_string(p.norm_tol) + ")");
        }
        return TBPM_OK;
    }
    if (corr_mean)
        sample_mean(corr_all, R, nt1, false, corr_mean);
    for (size_t r = 0; r < R; ++r)
        for (size_t k2 = 0; k2 < nt1; ++k2) {
            if (corr) {
                corr[(r * nt1 + k2) * 2] = corr_all[(k2 * R + r) * 2];
                corr[(r * nt1 + k2) * 2 + 1] = corr_all[(k2 * R + r) * 2 + 1];
            }
            if (norms)
                norms[r * nt1 + k2] = norms_all[k2 * R + r];
        }
    if (ldos && !sites.empty()) {
        const size_t cnt = sites.size() * nt1 * 2;
        if (hipMemcpy(ldos, site_dev, cnt * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(TBPM_ERR_HIP, "copy of the LDOS correlation failed");
        const double scale = (double)ham->n / (double)R;
        for (size_t i = 0; i < cnt; ++i)
            ldos[i] *= scale;
    }
    if (p.norm_tol > 0.0) {
        // the vectors whose blocks ran (all of them unless the run stopped early)
        for (size_t i = 0; i < R * nt1; ++i) {
            const size_t kk = i / R, rr = i % R;
            if (rr >= (size_t)rows_closed)
                continue;
            const double d = std::fabs(norms_all[i] - 1.0);
            if (!(d <= p.norm_tol)) {
                return fail(TBPM_ERR_DIVERGED, "norm of vector " + std::to_string(rr) + " at step " +
                                                   std::to_string(kk) + " is " + std::to_string(norms_all[i]) +
                                                   " (tolerance " + std::to_string(p.norm_tol) + ")");
            }
        }
    }
    return TBPM_OK;
}

}  // namespace tbpm
