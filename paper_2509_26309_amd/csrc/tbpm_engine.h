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
    void *vf = nullptr;                 // the seventh vector of pairs that straddle time steps
    bool pairs = false;                 // patch-reordered H, one vector per block
    // forward pairs straddling time steps (one vector, an even number of
    // series terms): a step whose successor is in the same block starts with
    // a pair of its terms 1 and 2 and ends with a pair of its last term and
    // the next step's term 1; that next step then runs its terms 2..M-1 in
    // pairs.  first_done: the previous step's last launch applied this step's
    // term 1.  Roles: psi(t_k) in P, Q and O the first two other vectors.
    bool cross = false;
    bool first_done = false;
    bool clenshaw = false;              // series by the backward recurrence (TBPM_SERIES_CLENSHAW)
    double *partials = nullptr;
    int max_grid = 8;
    double *corr_dev = nullptr;      // [N_t+1][bmax] complex
    int32_t *div_flag = nullptr;     // device: set by the reductions when a norm leaves norm_tol
    int32_t *div_host = nullptr;     // pinned copy of div_flag, read after a chunk completes
    int rows_closed = 0;             // vectors whose block has been copied to the host
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

    // time steps replayed from HIP graphs: GRAPH_STEPS consecutive steps are
    // captured per block width and starting buffer roles, and replayed; the
    // step index of the correlation rows comes from a device counter (kstep).
    // Plain and single-term series return the roles after GRAPH_STEPS steps
    // (a multiple of their rotation period, 3), so one graph serves a block
    // width; pairs that straddle steps move psi(t) between the work vectors
    // and, for some series lengths, cycle through up to three role sets.
    static constexpr int GRAPH_STEPS = 6;
    static constexpr int MAX_GRAPHS = 3;
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        void *sP = nullptr, *sQ = nullptr, *sO = nullptr;   // roles at the first captured step
        void *eP = nullptr, *eQ = nullptr, *eO = nullptr;   // roles the last step leaves
        int64_t terms = 0;                                  // term launches in the graph
    };
    bool graph_mode = false;
    int32_t *kstep = nullptr;
    std::vector<StepGraph> graphs;   // all captured for block width graph_B
    int graph_B = 0;
    int find_graph() const;          // index of the graph for the current roles, or -1
    void drop_graphs();

    // kernel timing: when set, each step records 4 events from ctx->events
    bool profile = false;
    size_t ev_used = 0;
    std::vector<size_t> step_ev;     // first of 4 pool events per eagerly launched step
    std::vector<size_t> graph_ev;    // first of 2 pool events around each graph launch
    bool capturing = false;          // steps being captured: no events, launch counts to graph_terms
    int64_t graph_terms = 0;         // term launches in the graph being captured
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
    // divergence seen so far: enqueue a copy of the device flag (norm_tol > 0),
    // and read it once the stream has passed that copy
    tbpm_status queue_flag_read();
    bool flag_set() const { return div_host && *div_host != 0; }
    // records an error raised outside the job's own steps
    tbpm_status fail_with(tbpm_status s, const std::string &msg) { return fail(s, msg); }
    // finalise host results (LDOS scaling, sample average, divergence check);
    // stream must be idle.  Every output may be NULL.
    tbpm_status finish(double *corr, double *norms, double *ldos, double *corr_mean = nullptr);

  private:
    void spare_buffers(void *out[3]) const;   // the rotating vectors not in P, Q, O (fixed order)
    void set_roles(void *psi);                 // P = psi; Q, O = the first two other vectors
    tbpm_status emit_outputs();      // snapshots / quasi-eigenstate terms of psi(t_k) (in P)
    tbpm_status graph_steps();       // GRAPH_STEPS steps from a captured graph (captured first if needed)
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
// skip_first: term 1 (Q = (1/rho) H P, O = c_0 P + c_1 Q) is already in Q and O.
tbpm_status apply_series(const tbpm_ham *ham, hipStream_t st, const KernelShape &shape, bool pairs, bool clenshaw,
                         const double *c, int M, double rescale, const SeriesBufs &bf, bool dots, const void *psi0,
                         double *partials, int *nblk, SeriesProfile *prof, std::string &err,
                         bool skip_first = false);
// A time step of one vector on patch-reordered H whose successor follows it
// (forward recurrence, M even >= 6): a pair of terms 1 and 2 from P (p_1 to
// Q, p_2 to spare[0], the series to O), the pairs of terms 3..M-2, and a
// pair of term M-1 with the next step's term 1: psi(t + dt) to *Pn, its p_1
// to *Qn and c_0 psi + c_1 p_1 to *On, with the correlation partials of
// psi(t + dt) (one block per patch).  *On is `keep` when that vector is
// free for it, so that the roles of two steps return to where they began.
tbpm_status apply_series_cross(const tbpm_ham *ham, hipStream_t st, const double *c, int M, double rescale,
                               void *P, void *Q, void *O, void *const spare[3], void *keep, const void *psi0,
                               double *partials, SeriesProfile *prof, void **Pn, void **Qn, void **On,
                               std::string &err);

// chosen block width for `params` (power of two, 1..64); pairs_ok: the
// route may run complex64 blocks in fused pairs (the forward recurrence)
int choose_block(const tbpm_ham *ham, const tbpm_params *p, bool pairs_ok);
// the (first vector, width) blocks a request's vectors run in
std::vector<std::pair<int, int>> split_blocks(const tbpm_ham *ham, const tbpm_params *p, bool pairs_ok);
// blocks of B > 1 vectors of `ham` take fused pairs of terms (forward recurrence)
bool block_pairs(const tbpm_ham *ham, int B);
// staged_ok: the staged complex64 SpMM may be chosen (not with a patch list)
KernelShape choose_shape(const tbpm_ham *ham, int B, int num_cu, int lanes_per_row, bool staged_ok = true);

}  // namespace tbpm
