"""GPU parity of the Clenshaw series (TBPM_SERIES_CLENSHAW) against the oracle.

The context evaluates each time step's series by the backward recurrence
b_m = c_m psi + 2 (H/rho) b_m+1 - b_m+2, psi(t + dt) = c_0 psi + (H/rho) b_1
- b_2; the oracle keeps the paper's forward recurrence.  Both give the same
polynomial in H, so the tolerances are those of the forward path:
  FP64 (complex128):  max |C_gpu - C_oracle| <= 1e-10
  FP32 (complex64):   max |C_gpu - C_oracle| <= 1e-5
Covered: single products in place (CSR with every lanes-per-row, ELL, SpMM
blocks in both precisions), fused pairs on patch-reordered H (both patch
sizes), every schedule length (series of 5..9 and 17..20 terms), LDOS sites,
given states, the response steps, HIP-graph replay and the request server.
"""
import time

import numpy as np
import pytest

from tb_inputs import graphene, bilayer, square, honeycomb3, current_operator

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5


@pytest.fixture(scope="module")
def T():
    from paper_2509_26309_amd import tbpm
    return tbpm


@pytest.fixture(scope="module")
def ctx(T):
    c = T.Context(0)
    T.tbpm_ctx_set_series(c.handle, T.TBPM_SERIES_CLENSHAW)
    yield c
    c.close()


def _run(T, ctx, lat, *, rho, nt, R=1, seed=1, dtype=0, fmt=2, block=0, lpr=0, sites=None, flags=0, eps=1e-14):
    ham = ctx.build(lat, dtype=dtype, fmt=fmt, flags=flags)
    try:
        p, _ = T.make_params(rho, nt, R, block=block, seed=seed, sites=sites, lanes_per_row=lpr, bessel_eps=eps)
        out = T.tbpm_propagate_dos(ctx.handle, ham, p)
        out["info"] = T.tbpm_ham_info(ham)
    finally:
        T.tbpm_ham_destroy(ham)
    return out


def _oracle(orc, lat, *, rho, nt, R=1, seed=1, sites=None, eps=1e-14):
    _, per, norms, ld = orc.corr_dos(lat, rescale=rho, num_steps=nt, num_vectors=R, seed=seed, sites=sites, eps=eps)
    return per, norms, ld


def test_mode_switch(T, ctx):
    with pytest.raises(T.TBPMError) as ei:
        T.tbpm_ctx_set_series(ctx.handle, 2)
    assert ei.value.status == T.TBPM_ERR_ARG


@pytest.mark.parametrize("fmt,lpr", [(0, 1), (0, 4), (0, 16), (1, 1)])
@pytest.mark.parametrize("dtype", [0, 1])
def test_single_products(T, ctx, orc, fmt, lpr, dtype):
    lat = graphene(13, 11, disorder_w=1.0, seed=5)        # 286 rows: ragged tail in every tiling
    out = _run(T, ctx, lat, rho=9.0, nt=40, fmt=fmt, lpr=lpr, dtype=dtype)
    per, norms, _ = _oracle(orc, lat, rho=9.0, nt=40)
    assert out["info"]["format"] == fmt
    tol = TOL64 if dtype == 0 else TOL32
    assert np.abs(out["corr"] - per).max() <= tol
    assert np.abs(out["norms"] - norms).max() <= tol


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("block", [2, 4, 8, 16, 32, 64])
def test_blocks(T, ctx, orc, block, dtype):
    lat = bilayer(9, 7, disorder_w=1.0, seed=8)
    R = block + 3 if block < 64 else 64
    out = _run(T, ctx, lat, rho=9.0, nt=24, R=R, block=block, seed=77, dtype=dtype, fmt=T.TBPM_FMT_ELL)
    per, _, _ = _oracle(orc, lat, rho=9.0, nt=24, R=R, seed=77)
    assert np.abs(out["corr"] - per).max() <= (TOL64 if dtype == 0 else TOL32)


PATCH_CASES = [
    ("graphene_W1_c128", lambda: graphene(100, 90, disorder_w=1.0, seed=21), 9.0, 0, 3, 1, [0, 17, 9000]),
    ("bilayer_W1_c128", lambda: bilayer(48, 40, disorder_w=1.0, seed=22), 9.0, 0, 2, 1, None),
    ("honeycomb3_vac_c64", lambda: honeycomb3(60, vacancy_p=0.01, seed=23), 10.0, 1, 2, 1, [5, 4000]),
    ("square_nnn_c64_block4", lambda: square(70), 4.5, 1, 5, 4, None),
]


@pytest.mark.parametrize("layout", ["pairs", "large"])
@pytest.mark.parametrize("name,make,rho,dtype,R,block,sites", PATCH_CASES, ids=[c[0] for c in PATCH_CASES])
def test_patch_format(T, ctx, orc, name, make, rho, dtype, R, block, sites, layout):
    """Fused Clenshaw pairs for single vectors (1024- or 2048-row patches),
    single products for blocks."""
    lat = make()
    flags = {"pairs": 0, "large": T.TBPM_BUILD_LARGE_PATCHES}[layout]
    out = _run(T, ctx, lat, rho=rho, nt=48, R=R, block=block, seed=31, dtype=dtype, fmt=T.TBPM_FMT_PATCH,
               sites=sites, flags=flags)
    assert out["info"]["format"] == T.TBPM_FMT_PATCH
    per, norms, ld = _oracle(orc, lat, rho=rho, nt=48, R=R, seed=31, sites=sites)
    tol = TOL64 if dtype == 0 else TOL32
    assert np.abs(out["corr"] - per).max() <= tol
    assert np.abs(out["norms"] - norms).max() <= tol
    if sites is not None:
        assert np.abs(out["ldos"] - ld).max() <= (TOL64 if dtype == 0 else 10 * TOL32)


@pytest.mark.parametrize("fmt", [1, 3])
@pytest.mark.parametrize("eps,M", [(0.1, 5), (0.02, 6), (0.005, 7), (0.001, 8), (2e-4, 9), (1e-11, 17),
                                   (1e-12, 18), (1e-13, 19), (1e-14, 20)])
def test_schedule_lengths(T, ctx, orc, eps, M, fmt):
    """Every schedule: single products for M >= 5 (ELL); on patches the first
    pair, a single product when M - 5 is odd, the middle pairs and the last
    pair for M >= 6 (forward pairs below)."""
    lat = graphene(80, 70, disorder_w=1.0, seed=24)
    out = _run(T, ctx, lat, rho=9.0, nt=30, R=2, seed=5, fmt=fmt, eps=eps)
    assert out["info"]["format"] == fmt
    assert orc.coefficients(np.pi, eps).size == M
    per, _, _ = _oracle(orc, lat, rho=9.0, nt=30, R=2, seed=5, eps=eps)
    assert np.abs(out["corr"] - per).max() <= TOL64


def test_given_states_and_final(T, ctx, orc):
    lat = graphene(60, disorder_w=1.0, seed=3)
    ham = ctx.build(lat, fmt=T.TBPM_FMT_PATCH)
    try:
        rng = np.random.default_rng(4)
        psi = rng.normal(size=(2, lat.n)) + 1j * rng.normal(size=(2, lat.n))
        psi /= np.linalg.norm(psi, axis=1, keepdims=True)
        p, _ = T.make_params(9.0, 20, 2)
        out = T.tbpm_propagate_states(ctx.handle, ham, p, psi, keep_final=True)
    finally:
        T.tbpm_ham_destroy(ham)
    for r in range(2):
        ref = orc.propagate(lat, psi[r], rescale=9.0, num_steps=20, keep_final=True)
        assert np.abs(out["corr"][r] - ref.corr).max() <= TOL64
        assert np.abs(out["psi_final"][r] - ref.psi_final).max() <= TOL64


@pytest.mark.parametrize("fmt", [1, 3])
def test_response_steps(T, ctx, orc, fmt):
    lat = graphene(192, disorder_w=1.0, seed=2) if fmt == 3 else graphene(24, disorder_w=1.0, seed=2)
    J = current_operator(lat, (1, 0))
    ham = ctx.build(lat, fmt=fmt)
    oa = ob = None
    try:
        oa = ctx.operator(ham, J)
        ob = ctx.operator(ham, J)
        p, _ = T.make_params(9.0, 8, 1, seed=3)
        got = T.tbpm_response_corr(ctx.handle, ham, oa, ob, p, -0.4, 0.3)
        assert T.tbpm_ham_info(ham)["format"] == fmt
    finally:
        for h in (oa, ob):
            if h is not None:
                T.tbpm_ham_destroy(h)
        T.tbpm_ham_destroy(ham)
    ref = orc.response_corr(lat, orc.random_state(lat.n, 3, 0), J, J, rescale=9.0, num_steps=8, mu=-0.4, kT=0.3)
    assert np.abs(got[0] - ref).max() <= 1e-10 * 0.2


@pytest.mark.parametrize("fmt,mids", [(1, 16), (3, 7)])
def test_response_profiled_launch_counts(T, ctx, fmt, mids):
    """Kernel timing of the time steps (two series per step): per series 2
    launches in the first group (the first product and the one after it, or
    the first pair and the single product), `mids` middle launches (16 single
    products, or 7 pairs) and 1 last launch, counted by position with its time."""
    lat = graphene(192, disorder_w=1.0, seed=2) if fmt == 3 else graphene(24, disorder_w=1.0, seed=2)
    J = current_operator(lat, (1, 0))
    nt = 3
    ham = ctx.build(lat, fmt=fmt)
    oa = None
    T.tbpm_ctx_set_profiling(ctx.handle, True)
    try:
        oa = ctx.operator(ham, J)
        p, _ = T.make_params(9.0, nt, 1, seed=1)
        T.tbpm_response_corr(ctx.handle, ham, oa, oa, p, 0.0, 0.3)
        k = [T.tbpm_ctx_kernel_time(ctx.handle, i) for i in range(3)]
        assert T.tbpm_ham_info(ham)["format"] == fmt
    finally:
        T.tbpm_ctx_set_profiling(ctx.handle, False)
        if oa is not None:
            T.tbpm_ham_destroy(oa)
        T.tbpm_ham_destroy(ham)
    series = 2 * nt
    assert [n for _, n in k] == [2 * series, mids * series, series]
    assert all(ms > 0 for ms, _ in k)


def test_graph_replay_bitwise(T, ctx, orc):
    """Captured steps replay the Clenshaw launches exactly (eager vs graph)."""
    lat = graphene(40, disorder_w=1.0, seed=6)
    ham = ctx.build(lat)
    try:
        res = {}
        for mode in (0, 2):
            T.tbpm_ctx_set_graphs(ctx.handle, mode)
            before = T.tbpm_ctx_graph_replays(ctx.handle)
            p, _ = T.make_params(9.0, 30, 3, block=1, seed=9)
            res[mode] = T.tbpm_propagate_dos(ctx.handle, ham, p)
            res[mode]["replays"] = T.tbpm_ctx_graph_replays(ctx.handle) - before
    finally:
        T.tbpm_ctx_set_graphs(ctx.handle, 1)
        T.tbpm_ham_destroy(ham)
    assert res[0]["replays"] == 0 and res[2]["replays"] > 0
    assert np.array_equal(res[0]["corr"], res[2]["corr"])
    per, _, _ = _oracle(orc, lat, rho=9.0, nt=30, R=3, seed=9)
    assert np.abs(res[2]["corr"] - per).max() <= TOL64


def test_server_alone_and_mixed(T, ctx):
    """Server requests take the context's series mode; results equal the
    direct call bit for bit, alone and in a mix."""
    lats = [graphene(30, disorder_w=1.0, seed=1), square(40), graphene(192, disorder_w=1.0, seed=2)]
    hams = [ctx.build(l) for l in lats]
    try:
        direct = []
        for h in hams:
            p, _ = T.make_params(9.0, 20, 2, seed=4)
            direct.append(T.tbpm_propagate_dos(ctx.handle, h, p)["corr"])
        srv = T.tbpm_server_create(ctx.handle, 8 << 30, 4)
        try:
            tickets = []
            for h in hams:
                p, _ = T.make_params(9.0, 20, 2, seed=4)
                tickets.append(T.tbpm_submit(srv, h, p))
            for t, ref in zip(tickets, direct):
                t0 = time.time()
                while True:
                    st, got, _, _ = T.tbpm_poll(srv, t, 2, 20)
                    if st != T.TBPM_PENDING:
                        break
                    assert time.time() - t0 < 60.0, "request still pending"
                    time.sleep(0.002)
                assert st == T.TBPM_OK
                assert np.array_equal(got, ref)
        finally:
            T.tbpm_server_destroy(srv)
    finally:
        for h in hams:
            T.tbpm_ham_destroy(h)


def test_moments_do_not_depend_on_the_series_mode(T, ctx):
    """The Chebyshev moments always use the forward recurrence (they need every
    p_m): bitwise the same on a Clenshaw context as on a forward one."""
    lat = graphene(192, disorder_w=1.0, seed=2)
    ham = ctx.build(lat)
    try:
        p, _ = T.make_params(9.0, 0, 1, seed=3)
        a = T.tbpm_chebyshev_moments(ctx.handle, ham, p, 101)
        T.tbpm_ctx_set_series(ctx.handle, T.TBPM_SERIES_FORWARD)
        try:
            b = T.tbpm_chebyshev_moments(ctx.handle, ham, p, 101)
        finally:
            T.tbpm_ctx_set_series(ctx.handle, T.TBPM_SERIES_CLENSHAW)
    finally:
        T.tbpm_ham_destroy(ham)
    assert np.array_equal(a, b)
