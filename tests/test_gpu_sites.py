"""GPU parity of the exact per-site LDOS path: site-localised initial states
e_i, through both routes (propagation: C_i(t) = <i|e^{-iHt}|i>; moments:
mu_m = <i|T_m(H/rho)|i>), against the oracle run on the same states, and
against the trace identity sum_i mu_m(i) = sum_n T_m(E_n / rho).
Tolerances as for random states: complex128 1e-10, complex64 1e-5."""
import numpy as np
import pytest

from tb_inputs import graphene, bilayer, honeycomb3, square, state_from_sites, sample_sites

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-5}


@pytest.fixture(scope="module")
def T():
    from paper_2509_26309_amd import tbpm
    return tbpm


@pytest.fixture(scope="module")
def ctx(T):
    c = T.Context(0)
    yield c
    c.close()


def _ham(T, ctx, lat, dtype, fmt, fn):
    ham = ctx.build(lat, dtype=dtype, fmt=fmt)
    try:
        return fn(ham), T.tbpm_ham_info(ham)
    finally:
        T.tbpm_ham_destroy(ham)


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("fmt,block", [(0, 1), (0, 4), (1, 8), (1, 16), (2, 1), (2, 16)])
def test_site_moments(T, ctx, orc, fmt, block, dtype):
    lat = graphene(192, disorder_w=1.0, seed=2) if fmt == 2 else honeycomb3(12, vacancy_p=0.03, seed=4)
    sites = sample_sites(lat.n, 19, 7)                    # ragged over the blocks
    p, _ = T.make_params(10.0, 0, 1, block=block)
    mu, info = _ham(T, ctx, lat, dtype, fmt, lambda h: T.tbpm_site_moments(ctx.handle, h, p, sites, 121))
    if fmt == 2:
        assert info["format"] == T.TBPM_FMT_PATCH
    ref = np.stack([orc.moments(lat, state_from_sites(lat.n, [i]), rescale=10.0, num_moments=121) for i in sites])
    assert np.abs(mu - ref).max() <= TOL[dtype]


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("fmt,block", [(0, 2), (1, 8), (2, 1)])
def test_propagate_sites(T, ctx, orc, fmt, block, dtype):
    lat = graphene(192, disorder_w=1.0, seed=2) if fmt == 2 else bilayer(6, disorder_w=1.0, seed=1)
    sites = sample_sites(lat.n, 9, 3)
    nt = 48
    p, _ = T.make_params(9.0, nt, 1, block=block)
    out, _ = _ham(T, ctx, lat, dtype, fmt, lambda h: T.tbpm_propagate_sites(ctx.handle, h, p, sites))
    ref = np.stack([orc.propagate(lat, state_from_sites(lat.n, [i]), rescale=9.0, num_steps=nt).corr
                    for i in sites])
    assert np.abs(out["corr"] - ref).max() <= TOL[dtype]
    assert np.abs(out["norms"] - 1.0).max() <= TOL[dtype]


def test_site_moments_trace_identity(T, ctx):
    """Summed over every site the local moments give the trace sum_n T_m(E_n/rho)."""
    lat = bilayer(3, disorder_w=1.0, seed=5)
    p, _ = T.make_params(9.0, 0, 1, block=8)
    mu, _ = _ham(T, ctx, lat, 0, 1, lambda h: T.tbpm_site_moments(ctx.handle, h, p, np.arange(lat.n), 200))
    e = np.linalg.eigvalsh(lat.to_dense())
    ref = np.array([np.cos(m * np.arccos(e / 9.0)).sum() for m in range(200)])
    assert np.abs(mu.sum(axis=0) - ref).max() <= 1e-10 * lat.n


def test_square_single_site_closed_form(T, ctx):
    """Square lattice NN: C_0(t) = [(1/L) sum_q exp(-2 i t_h cos q t)]^2 for every site."""
    from tb_inputs import supercell, square_cell
    L, th, rho, nt = 32, -1.0, 4.5, 60
    lat = supercell(square_cell(th, 0.0), L, L)
    p, _ = T.make_params(rho, nt, 1, block=4)
    out, _ = _ham(T, ctx, lat, 0, 0, lambda h: T.tbpm_propagate_sites(ctx.handle, h, p, [0, 5, 333, 1023]))
    t = np.arange(nt + 1) * np.pi / rho
    q = 2 * np.pi * np.arange(L) / L
    ring = np.exp(-2j * th * np.outer(t, np.cos(q))).mean(axis=1)
    assert np.abs(out["corr"] - ring[None, :] ** 2).max() <= 1e-12


def test_site_errors(T, ctx):
    lat = graphene(6)
    ham = ctx.build(lat)
    try:
        p, _ = T.make_params(9.0, 4, 1)
        with pytest.raises(T.TBPMError):
            T.tbpm_propagate_sites(ctx.handle, ham, p, [lat.n])
        with pytest.raises(T.TBPMError):
            T.tbpm_site_moments(ctx.handle, ham, p, [-1], 8)
        with pytest.raises(T.TBPMError):
            T.tbpm_site_moments(ctx.handle, ham, p, [], 8)
    finally:
        T.tbpm_ham_destroy(ham)
