"""Time steps replayed from HIP graphs give the same results, bit for bit, as
the same kernels launched one by one: per-step launches with a fixed-order
reduction whose row index comes from a device counter.  Each case runs with
graphs off, then on (several replays per call, and calls repeated with eager
work in between), and compares every value exactly; one case also against the
oracle."""
import numpy as np
import pytest

from tb_inputs import graphene, bilayer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2509_26309_amd import tbpm
    return tbpm


@pytest.fixture(scope="module")
def ctx(T):
    c = T.Context(0)
    yield c
    T.tbpm_ctx_set_graphs(c.handle, 1)
    c.close()


def _run(T, ctx, ham, *, rho, nt, R, block, seed, mode):
    T.tbpm_ctx_set_graphs(ctx.handle, mode)
    before = T.tbpm_ctx_graph_replays(ctx.handle)
    p, _ = T.make_params(rho, nt, R, block=block, seed=seed)
    out = T.tbpm_propagate_dos(ctx.handle, ham, p)
    return out, T.tbpm_ctx_graph_replays(ctx.handle) - before


CASES = [
    ("csr_c128", lambda: graphene(13, 11, disorder_w=1.0, seed=5), 0, 0, 1, 1, 40),
    ("ell_c128", lambda: graphene(13, 11, disorder_w=1.0, seed=5), 1, 0, 1, 1, 13),
    ("ell_c64_blocks", lambda: bilayer(9, disorder_w=1.0, seed=3), 1, 1, 19, 16, 30),
    ("patch_pairs", lambda: graphene(192, disorder_w=1.0, seed=2), 2, 0, 1, 1, 25),
]


@pytest.mark.parametrize("name,make,fmt,dtype,R,block,nt", CASES, ids=[c[0] for c in CASES])
def test_graph_replay_is_bitwise_eager(T, ctx, name, make, fmt, dtype, R, block, nt):
    lat = make()
    ham = ctx.build(lat, dtype=dtype, fmt=fmt)
    try:
        eager, n0 = _run(T, ctx, ham, rho=9.0, nt=nt, R=R, block=block, seed=4, mode=0)
        assert n0 == 0
        for rep in range(2):
            graph, n1 = _run(T, ctx, ham, rho=9.0, nt=nt, R=R, block=block, seed=4, mode=2)
            blocks = [16, 2, 1] if R == 19 else [1]
            assert n1 == len(blocks) * (nt // 6)
            assert np.array_equal(graph["corr"], eager["corr"])
            assert np.array_equal(graph["norms"], eager["norms"])
            # eager work between the replays
            _run(T, ctx, ham, rho=9.0, nt=7, R=1, block=1, seed=9, mode=0)
    finally:
        T.tbpm_ham_destroy(ham)


@pytest.mark.parametrize("eps,M", [(1e-12, 18), (1e-14, 20)])
def test_graph_replay_cross_step_pairs_any_role_cycle(T, ctx, orc, eps, M):
    """Pairs that straddle time steps move psi(t) between the work vectors; with
    an odd number of middle pairs (M = 18) six steps do not bring the buffer
    roles back, and a second graph is captured from the roles the first one
    leaves.  Every chunk of six steps replays; bitwise against eager launches,
    and against the oracle."""
    assert orc.coefficients(np.pi, eps).size == M
    lat = graphene(80, 70, disorder_w=1.0, seed=24)
    ham = ctx.build(lat, fmt=2)
    try:
        def run(mode):
            T.tbpm_ctx_set_graphs(ctx.handle, mode)
            before = T.tbpm_ctx_graph_replays(ctx.handle)
            p, _ = T.make_params(9.0, 40, 2, block=1, seed=5, bessel_eps=eps)
            out = T.tbpm_propagate_dos(ctx.handle, ham, p)
            return out, T.tbpm_ctx_graph_replays(ctx.handle) - before
        eager, n0 = run(0)
        graph, n1 = run(2)
        assert n0 == 0 and n1 == 2 * (40 // 6)
        assert np.array_equal(graph["corr"], eager["corr"])
        assert np.array_equal(graph["norms"], eager["norms"])
        mean, per, _, _ = orc.corr_dos(lat, rescale=9.0, num_steps=40, num_vectors=2, seed=5, eps=eps)
        assert np.abs(graph["corr"] - per).max() <= 1e-10
    finally:
        T.tbpm_ham_destroy(ham)


def test_graph_against_oracle_and_profiled(T, ctx, orc):
    lat = graphene(64)
    ham = ctx.build(lat, fmt=0)
    try:
        T.tbpm_ctx_set_profiling(ctx.handle, True)
        out, n = _run(T, ctx, ham, rho=9.0, nt=256, R=1, block=1, seed=1, mode=1)
        ms, launches = T.tbpm_ctx_kernel_time(ctx.handle, 1)
        T.tbpm_ctx_set_profiling(ctx.handle, False)
        assert n == 256 // 6
        assert ms > 0 and launches >= 256 // 6 * 6 * 18
        mean, per, norms, _ = orc.corr_dos(lat, rescale=9.0, num_steps=256, num_vectors=1, seed=1)
        assert np.abs(out["corr"] - per).max() <= 1e-10
    finally:
        T.tbpm_ham_destroy(ham)


def test_graphs_off_for_per_step_outputs(T, ctx):
    lat = graphene(10)
    ham = ctx.build(lat)
    try:
        T.tbpm_ctx_set_graphs(ctx.handle, 2)
        before = T.tbpm_ctx_graph_replays(ctx.handle)
        p, keep = T.make_params(9.0, 24, 2, sites=[0, 5])
        T.tbpm_propagate_dos(ctx.handle, ham, p)
        p1, _ = T.make_params(9.0, 24, 1)
        T.tbpm_quasi_eigenstates(ctx.handle, ham, p1, [0.0])
        assert T.tbpm_ctx_graph_replays(ctx.handle) == before
        with pytest.raises(T.TBPMError):
            T.tbpm_ctx_set_graphs(ctx.handle, 3)
    finally:
        T.tbpm_ctx_set_graphs(ctx.handle, 1)
        T.tbpm_ham_destroy(ham)


def test_graph_replays_with_chunked_requests(T, ctx):
    """The server advances a request a few steps at a time; eager steps at a
    chunk's end rotate the buffer roles, and a replay must wait until they are
    back to the captured ones.  Results equal the eager run bit for bit."""
    from tb_inputs import square
    import time
    lat = square(20)
    ham = ctx.build(lat, dtype=1)
    try:
        eager, _ = _run(T, ctx, ham, rho=4.5, nt=200, R=2, block=0, seed=16, mode=0)
        T.tbpm_ctx_set_graphs(ctx.handle, 1)
        before = T.tbpm_ctx_graph_replays(ctx.handle)
        srv = T.tbpm_server_create(ctx.handle, 1 << 28, 1)
        try:
            p, _ = T.make_params(4.5, 200, 2, seed=16)
            t = T.tbpm_submit(srv, ham, p)
            while True:
                st, corr, _tm, _ = T.tbpm_poll(srv, t, 2, 200)
                if st != T.TBPM_PENDING:
                    break
                time.sleep(0.01)
        finally:
            T.tbpm_server_destroy(srv)
        assert st == T.TBPM_OK
        assert T.tbpm_ctx_graph_replays(ctx.handle) > before
        assert np.array_equal(corr, eager["corr"])
    finally:
        T.tbpm_ham_destroy(ham)


def test_graph_replay_block_pairs_bitwise_eager(T, ctx, orc):
    """Complex64 blocks in fused pairs (patch format): replayed steps equal the
    eager launches bit for bit, and both match the oracle."""
    lat = bilayer(128, disorder_w=1.0, seed=3)
    ham = ctx.build(lat, dtype=1, fmt=2)
    R, nt = 11, 13                                   # blocks of 8, 2, 1
    try:
        assert T.tbpm_ham_fused_pairs(ham, 8)
        eager, n0 = _run(T, ctx, ham, rho=9.0, nt=nt, R=R, block=8, seed=6, mode=0)
        assert n0 == 0
        for rep in range(2):
            graph, n1 = _run(T, ctx, ham, rho=9.0, nt=nt, R=R, block=8, seed=6, mode=2)
            assert n1 == 3 * (nt // 6)
            assert np.array_equal(graph["corr"], eager["corr"])
            assert np.array_equal(graph["norms"], eager["norms"])
            _run(T, ctx, ham, rho=9.0, nt=7, R=1, block=1, seed=9, mode=0)
    finally:
        T.tbpm_ctx_set_graphs(ctx.handle, 1)
        T.tbpm_ham_destroy(ham)
    _, per, _, _ = orc.corr_dos(lat, rescale=9.0, num_steps=nt, num_vectors=R, seed=6)
    assert np.abs(eager["corr"] - per).max() <= 1e-5
