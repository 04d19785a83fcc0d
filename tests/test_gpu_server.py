"""GPU tests of the request server (continuous batching).

Each request's result must equal the same request run alone through
tbpm_propagate_dos (bit for bit: same kernels, launch shapes and reduction
order), and agree with the oracle within the path's tolerance.
"""
import time

import numpy as np
import pytest

from tb_inputs import graphene, square

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2509_26309_amd import tbpm
    return tbpm


@pytest.fixture(scope="module")
def ctx(T):
    c = T.Context(0)
    yield c
    c.close()


def _wait(T, srv, ticket, R, nt, timeout=60.0):
    t0 = time.time()
    while True:
        st, corr, tm, mean = T.tbpm_poll(srv, ticket, R, nt)
        if st != T.TBPM_PENDING:
            return st, corr, tm, mean
        if time.time() - t0 > timeout:
            raise TimeoutError(f"ticket {ticket} still pending")
        time.sleep(0.002)


REQS = [
    # (lattice maker, rho, R, N_t, dtype, seed)
    (lambda: graphene(40, disorder_w=1.0, seed=1), 9.0, 3, 64, 0, 11),
    (lambda: square(50), 4.5, 5, 40, 1, 12),
    (lambda: graphene(64), 9.0, 1, 128, 0, 13),
    (lambda: square(33), 4.5, 16, 32, 0, 14),
    (lambda: graphene(30, 50), 9.0, 8, 48, 1, 15),
    (lambda: square(20), 4.5, 2, 200, 1, 16),
    (lambda: graphene(200, disorder_w=0.5, seed=3), 9.0, 2, 40, 0, 17),      # patch format (fused pairs)
]


def test_mix_equals_alone(T, ctx, orc):
    lats = [m() for (m, *_rest) in REQS]
    hams = []
    alone = []
    for lat, (_, rho, R, nt, dt, seed) in zip(lats, REQS):
        h = ctx.build(lat, dtype=dt)
        hams.append(h)
        p, _ = T.make_params(rho, nt, R, seed=seed)
        o = T.tbpm_propagate_dos(ctx.handle, h, p)
        alone.append((o["corr"], o["corr_mean"]))
    srv = T.tbpm_server_create(ctx.handle, 1 << 30, 3)
    try:
        tickets = []
        for h, (_, rho, R, nt, dt, seed) in zip(hams, REQS):
            p, _ = T.make_params(rho, nt, R, seed=seed)
            tickets.append(T.tbpm_submit(srv, h, p))
        results = [_wait(T, srv, t, R, nt) for t, (_, _, R, nt, _, _) in zip(tickets, REQS)]
    finally:
        T.tbpm_server_destroy(srv)
    for (st, corr, tm, mean), (ref, ref_mean), lat, (_, rho, R, nt, dt, seed) in zip(results, alone, lats, REQS):
        assert st == T.TBPM_OK
        assert np.array_equal(corr, ref)
        assert np.array_equal(mean, ref_mean)       # the sample average, served and alone
        assert tm[0] <= tm[1] <= tm[2]
    assert T.tbpm_ham_info(hams[-1])["format"] == T.TBPM_FMT_PATCH
    # spot check three requests against the oracle
    for i in (0, 1, len(REQS) - 1):
        _, rho, R, nt, dt, seed = REQS[i]
        ref_mean, per, _, _ = orc.corr_dos(lats[i], rescale=rho, num_steps=nt, num_vectors=R, seed=seed)
        tol = 1e-10 if dt == 0 else 1e-5
        assert np.abs(results[i][1] - per).max() <= tol
        assert np.abs(results[i][3] - ref_mean).max() <= tol
    # the mix overlapped: with three slots, some request was admitted before another finished
    spans = sorted((tm[1], tm[2]) for (_, _, tm, _) in results)
    assert any(spans[j + 1][0] < spans[j][1] for j in range(len(spans) - 1))
    for h in hams:
        T.tbpm_ham_destroy(h)


def test_budget_slots_cancel(T, ctx):
    lat = graphene(32)
    h = ctx.build(lat)
    p, _ = T.make_params(9.0, 64, 2, seed=1)
    fp = T.tbpm_footprint(h, p)
    # budget for exactly one request at a time
    srv = T.tbpm_server_create(ctx.handle, fp + fp // 2, 8)
    try:
        big, _ = T.make_params(9.0, 64, 64, seed=1)
        with pytest.raises(T.TBPMError) as ei:
            T.tbpm_submit(srv, h, big)
        assert ei.value.status == T.TBPM_ERR_TOO_LARGE
        t1 = T.tbpm_submit(srv, h, p)
        t2 = T.tbpm_submit(srv, h, p)
        t3 = T.tbpm_submit(srv, h, p)
        T.tbpm_cancel(srv, t3)
        s1, c1, m1, _ = _wait(T, srv, t1, 2, 64)
        s2, c2, m2, _ = _wait(T, srv, t2, 2, 64)
        s3, _, _, _ = _wait(T, srv, t3, 2, 64)
        assert s1 == s2 == T.TBPM_OK and s3 == T.TBPM_ERR_CANCELLED
        assert m2[1] >= m1[2]                 # admitted only after the first one finished
        assert np.array_equal(c1, c2)
        # output buffers smaller than the request are refused before anything is written
        for R_, nt_ in ((1, 64), (2, 63)):
            with pytest.raises(T.TBPMError) as ei:
                T.tbpm_poll(srv, t1, R_, nt_)
            assert ei.value.status == T.TBPM_ERR_ARG
        with pytest.raises(T.TBPMError) as ei:
            T.tbpm_poll(srv, 987654, 1, 1)
        assert ei.value.status == T.TBPM_ERR_UNKNOWN
    finally:
        T.tbpm_server_destroy(srv)
    T.tbpm_ham_destroy(h)


def test_large_fp32_requests_against_bloch_sums(T, ctx, orc):
    """Served complex64 requests of about 10^6 orbitals (the serving mix spans
    10^4..10^7, all clean and periodic), each vector pinned against its exact
    Bloch sum; a small complex128 request runs in the same mix."""
    from bloch import corr_graphene, corr_square
    reqs = [
        # (lattice, L, vectors, steps, dtype, seed)
        ("graphene", 724, 2, 128, T.TBPM_C64, 41),
        ("square_nnn", 1024, 3, 96, T.TBPM_C64, 42),
        ("graphene", 40, 2, 64, T.TBPM_C128, 43),
    ]
    lats, hams, tickets = [], [], []
    srv = T.tbpm_server_create(ctx.handle, 16 << 30, 3)
    try:
        for kind, L, R, nt, dt, seed in reqs:
            lat = graphene(L) if kind == "graphene" else square(L)
            lats.append(lat)
            h = ctx.build(lat, dtype=dt)
            hams.append(h)
            p, _ = T.make_params(9.0 if kind == "graphene" else 4.5, nt, R, seed=seed)
            tickets.append(T.tbpm_submit(srv, h, p))
        results = [_wait(T, srv, t, R, nt, timeout=120.0) for t, (_, _, R, nt, _, _) in zip(tickets, reqs)]
    finally:
        T.tbpm_server_destroy(srv)
        for h in hams:
            T.tbpm_ham_destroy(h)
    for (kind, L, R, nt, dt, seed), lat, (st, corr, tm, mean) in zip(reqs, lats, results):
        assert st == T.TBPM_OK
        rho = 9.0 if kind == "graphene" else 4.5
        times = np.arange(nt + 1) * np.pi / rho
        tol = 1e-5 if dt == T.TBPM_C64 else 1e-10
        for r in range(R):
            psi0 = orc.random_state(lat.n, seed, r)
            ref = corr_graphene(psi0, L, L, -2.7, times) if kind == "graphene" else \
                corr_square(psi0, L, L, -1.0, 0.1, times)
            err = float(np.abs(corr[r] - ref).max())
            print(f"served {kind} {lat.n} orbitals dtype={dt} vector {r}: max|dC| vs Bloch sum {err:.3e}",
                  flush=True)
            assert err <= tol


def test_diverging_request_frees_its_slot_early(T, ctx):
    """A request whose norms leave norm_tol (forced from the host with a
    tolerance no norm meets) is stopped at the first chunk that shows it, not
    run to the end: its service time is a fraction of the same request's
    without the check."""
    lat = graphene(64)
    h = ctx.build(lat)
    srv = T.tbpm_server_create(ctx.handle, 1 << 30, 2)
    try:
        p_ok, _ = T.make_params(9.0, 3000, 1, seed=3)
        p_bad, _ = T.make_params(9.0, 3000, 1, seed=3, norm_tol=1e-300)
        t_ok = T.tbpm_submit(srv, h, p_ok)
        s_ok, _, tm_ok, _ = _wait(T, srv, t_ok, 1, 3000)
        t_bad = T.tbpm_submit(srv, h, p_bad)
        s_bad, corr, tm_bad, _ = _wait(T, srv, t_bad, 1, 3000)
    finally:
        T.tbpm_server_destroy(srv)
        T.tbpm_ham_destroy(h)
    assert s_ok == T.TBPM_OK and s_bad == T.TBPM_ERR_DIVERGED and corr is None
    svc_ok, svc_bad = tm_ok[2] - tm_ok[1], tm_bad[2] - tm_bad[1]
    print(f"service: full run {svc_ok:.3f} s, stopped run {svc_bad:.3f} s", flush=True)
    assert svc_bad < 0.5 * svc_ok
