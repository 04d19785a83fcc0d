// Propagation engine: one request (a Hamiltonian, parameters and R vectors)
// advanced block by block and step by step on one HIP stream.  Used
// synchronously by tbpm_propagate_dos / tbpm_propagate_states and
// incrementally by the request server.
#pragma once

#include <string>
#include <vector>

#include "tbpm_internal.h"

namespace tbpm {

struct Job {
    tbpm_ctx *ctx = nullptr;
    const tbpm_ham *ham = nullptr;
    tbpm_params p{};
    std::vector<int64_t> sites;      // LDOS sites (host copy)
    hipStream_t st = nullptr;

    // Chebyshev series
    std::vector<double> coeff;       // interleaved complex, M entries
    int M = 0;

    // device buffers, sized for the widest block
    int bmax = 1;
    size_t elem = 16;                // bytes per complex element
    void *psi0 = nullptr, *va = nullptr, *vb = nullptr, *vc = nullptr;
    void *vd = nullptr, *ve = nullptr;  // out-of-place targets of fused term pairs
    bool pairs = false;                 // patch-reordered H, one vector per block
    bool clenshaw = false;              // series by the backward recurrence (TBPM_SERIES_CLENSHAW)
    double *partials = nullptr;
    int max_grid = 8;
    double *corr_dev = nullptr;      // [N_t+1][bmax] complex
    double *norms_dev = nullptr;     // [N_t+1][bmax]
    double *site_dev = nullptr;      // [S][N_t+1] complex
    int64_t *sites_dev = nullptr;
    double *states_dev = nullptr;    // staging for given initial / final states [bmax][n] complex

    // host results (pinned), [N_t+1][R]; each block's columns are copied in
    // with one strided copy when the block closes
    double *corr_all = nullptr;      // complex
    double *norms_all = nullptr;

    // allocation-free mode: every device buffer is carved from the caller's
    // [arena, arena + arena_bytes) (never freed here), no HIP graphs, no
    // events, no pinned host memory; each vector's C(t) (and norms) is copied
    // straight into the caller's host rows direct_corr [R][N_t+1] complex
    // (direct_norms [R][N_t+1], optional)
    char *arena = nullptr;
    size_t arena_bytes = 0;
    size_t arena_used = 0;
    double *direct_corr = nullptr;
    double *direct_norms = nullptr;
    // device bytes the allocation-free mode carves (256-byte aligned buffers)
    size_t arena_need() const;

    // vector blocks: (first vector offset, width)
    std::vector<std::pair<int, int>> blocks;
    size_t cur_block = 0;
    bool block_open = false;
    int k = 0;                        // steps done in the open block
    void *P = nullptr, *Q = nullptr, *O = nullptr;
    KernelShape shape{};
    int dot_grid = 8;

    // site-localised initial states (tbpm_propagate_sites): vector r is
    // e_i with i = site_states[r] (original orbital index)
    std::vector<int64_t> site_states;
    // given initial states (tbpm_propagate_states), host complex [R][n]
    const double *given_states = nullptr;
    double *final_states = nullptr;

    // one-vector outputs: snapshots psi(t_k) at listed steps (host complex
    // [S][n]) and quasi-eigenstates sum_k w_k e^{i E_j t_k} psi(t_k) (host
    // complex [E][n], accumulated on the device in FP64)
    std::vector<int32_t> snap_steps;
    double *snaps = nullptr;
    std::vector<double> qe_energies;
    double *qe_host = nullptr;
    double *qe_dev = nullptr;

    std::string error;

    // time steps replayed from a HIP graph: GRAPH_STEPS consecutive steps are
    // captured once per block width and replayed; the step index of the
    // correlation rows comes from a device counter (kstep)
    static constexpr int GRAPH_STEPS = 6;   // a multiple of the buffer rotation period (3)
    bool graph_mode = false;
    int32_t *kstep = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_B = 0;
    void *cap_P = nullptr, *cap_Q = nullptr, *cap_O = nullptr;   // buffer roles the graph was captured with

    // kernel timing: when set, each step records 4 events from ctx->events
    bool profile = false;
    size_t ev_used = 0;
    std::vector<size_t> step_ev;     // first of 4 pool events per eagerly launched step
    std::vector<size_t> graph_ev;    // first of 2 pool events around each graph launch
    bool capturing = false;          // steps being captured: no events, launch counts to graph_terms
    int64_t graph_terms = 0;         // term launches in one graph
    int64_t prof_launch[3] = {0, 0, 0};
    tbpm_status collect_profile();   // after the stream has drained

    ~Job();
    // validate, compute coefficients and the block plan; no device work
    tbpm_status setup(tbpm_ctx *c, const tbpm_ham *h, const tbpm_params *prm, hipStream_t stream);
    // device bytes allocate() will take
    size_t footprint() const;
    tbpm_status allocate();
    void release();
    // enqueue up to max_steps time steps (opening/closing blocks as needed);
    // returns TBPM_OK when every block has been enqueued, TBPM_PENDING otherwise
    tbpm_status advance(int max_steps);
    bool all_enqueued() const { return cur_block >= blocks.size() && !block_open; }
    // records an error raised outside the job's own steps
    tbpm_status fail_with(tbpm_status s, const std::string &msg) { return fail(s, msg); }
    // finalise host results (LDOS scaling, sample average, divergence check);
    // stream must be idle.  Every output may be NULL.
    tbpm_status finish(double *corr, double *norms, double *ldos, double *corr_mean = nullptr);

  private:
    tbpm_status emit_outputs();      // snapshots / quasi-eigenstate terms of psi(t_k) (in P)
    tbpm_status graph_steps();       // GRAPH_STEPS steps from the captured graph
    tbpm_status open_block();
    tbpm_status close_block();
    tbpm_status step();
    tbpm_status fail(tbpm_status s, const std::string &msg);
};

// Buffers of one series application: input P (may be overwritten), output O,
// scratch Q, and S1, S2 (used by fused pairs of terms).
struct SeriesBufs {
    void *P, *Q, *O, *S1, *S2;
};
// Optional kernel timing: events recorded after the first term (ev[1]),
// before the last launch (ev[2]) and after it (ev[3]); launch counts per kind.
struct SeriesProfile {
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    int64_t launches[3] = {0, 0, 0};
};
// O = sum_{m<M} c_m T_m(H/rho) P for a block of shape.B vectors, with the term
// kernels of the stored format (for B = 1 on patch-reordered H when `pairs`:
// fused pairs, or K-term groups of the forward recurrence).  clenshaw: the
// backward recurrence instead (single products when M >= 5; fused pairs when
// `pairs`, B = 1, M >= 6 and two terms per pass).  dots: the last launch also writes the per-block partials of
// <psi0|O> and <O|O> into `partials`; *nblk receives their count (-1: M = 2,
// none written).  c: M complex coefficients (interleaved).
tbpm_status apply_series(const tbpm_ham *ham, hipStream_t st, const KernelShape &shape, bool pairs, bool clenshaw,
                         const double *c, int M, double rescale, const SeriesBufs &bf, bool dots, const void *psi0,
                         double *partials, int *nblk, SeriesProfile *prof, std::string &err);

// chosen block width for `params` (power of two, 1..64)
int choose_block(const tbpm_ham *ham, const tbpm_params *p);
// staged_ok: the staged complex64 SpMM may be chosen (not with a patch list)
KernelShape choose_shape(const tbpm_ham *ham, int B, int num_cu, int lanes_per_row, bool staged_ok = true);

}  // namespace tbpm
