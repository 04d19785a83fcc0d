"""The value table of the patch format (one byte per entry indexing the few
distinct hoppings, the on-site energies per row under disorder) gives the
same results, bit for bit, as the same matrix stored with every value
(TBPM_BUILD_NO_VALUE_TABLE): the fused-pair kernel in every mode (forward
pairs with cross-step pairs, Clenshaw pairs, moments) and the staged
complex64 SpMM kernel (forward, Clenshaw, moments), in both precisions; and
against the oracle."""
from types import SimpleNamespace

import numpy as np
import pytest

from tb_inputs import graphene, bilayer, honeycomb3

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-10, 1e-5


@pytest.fixture(scope="module")
def T():
    from paper_2509_26309_amd import tbpm
    return tbpm


@pytest.fixture(scope="module")
def ctx(T):
    c = T.Context(0)
    yield c
    T.tbpm_ctx_set_series(c.handle, T.TBPM_SERIES_FORWARD)
    c.close()


def _complex_onsite(lat):
    """On-site energies with small imaginary parts (an absorbing potential): the
    per-row diagonal then keeps whole complex values."""
    rows = np.repeat(np.arange(lat.n), np.diff(lat.row_ptr))
    v = lat.val.copy()
    d = lat.col == rows
    v[d] = v[d] - 0.01j
    return SimpleNamespace(n=lat.n, row_ptr=lat.row_ptr, col=lat.col, val=v)


def _both(T, ctx, lat, dtype, run):
    """run(ham) on the matrix stored with and without the value table."""
    res = []
    for flags in (0, T.TBPM_BUILD_NO_VALUE_TABLE):
        ham = ctx.build(lat, dtype=dtype, fmt=T.TBPM_FMT_PATCH, flags=flags)
        try:
            assert T.tbpm_ham_info(ham)["format"] == T.TBPM_FMT_PATCH
            res.append((T.tbpm_ham_value_table(ham), run(ham)))
        finally:
            T.tbpm_ham_destroy(ham)
    (vt, a), (vt0, b) = res
    assert vt["entries"] > 0 and vt0["entries"] == 0
    return vt, a, b


CASES = [
    # name, lattice, dtype, rho, vectors, block, per-row diagonal (0: in the table, 1: complex, 2: real parts)
    ("graphene_disorder_c128", lambda: graphene(80, 70, disorder_w=1.0, seed=24), 0, 9.0, 2, 1, 2),
    ("graphene_complex_onsite_c128", lambda: _complex_onsite(graphene(80, 70, disorder_w=1.0, seed=24)), 0, 9.0,
     1, 1, 1),
    ("graphene_clean_c64", lambda: graphene(96), 1, 9.0, 1, 1, 0),
    ("bilayer_disorder_c64_b16", lambda: bilayer(128, disorder_w=1.0, seed=3), 1, 9.0, 16, 16, 2),
    ("bilayer_complex_onsite_c64_b8", lambda: _complex_onsite(bilayer(128, disorder_w=1.0, seed=3)), 1, 9.0, 8, 8,
     1),
    ("honeycomb3_vac_c64_b8", lambda: honeycomb3(190, vacancy_p=0.01, seed=5), 1, 10.0, 8, 8, 0),
]


@pytest.mark.parametrize("series", [0, 1], ids=["forward", "clenshaw"])
@pytest.mark.parametrize("name,make,dtype,rho,R,block,diag", CASES, ids=[c[0] for c in CASES])
def test_table_is_bitwise_the_stored_values(T, ctx, orc, name, make, dtype, rho, R, block, diag, series):
    lat = make()
    nt = 20
    T.tbpm_ctx_set_series(ctx.handle, series)

    def run(ham):
        p, _ = T.make_params(rho, nt, R, block=block, seed=7)
        return T.tbpm_propagate_dos(ctx.handle, ham, p)

    try:
        vt, a, b = _both(T, ctx, lat, dtype, run)
    finally:
        T.tbpm_ctx_set_series(ctx.handle, T.TBPM_SERIES_FORWARD)
    assert vt["per_row_diagonal"] == diag
    assert np.array_equal(a["corr"], b["corr"])
    assert np.array_equal(a["norms"], b["norms"])
    if diag != 1:                               # a non-Hermitian H is outside the oracle's propagator
        mean, per, norms, _ = orc.corr_dos(lat, rescale=rho, num_steps=nt, num_vectors=R, seed=7)
        assert np.abs(a["corr"] - per).max() <= (TOL64 if dtype == 0 else TOL32)


@pytest.mark.parametrize("name,make,dtype,rho,R,block,diag", CASES, ids=[c[0] for c in CASES])
def test_table_moments_bitwise(T, ctx, orc, name, make, dtype, rho, R, block, diag):
    lat = make()

    def run(ham):
        p, _ = T.make_params(rho, 0, R, block=block, seed=9)
        return T.tbpm_chebyshev_moments(ctx.handle, ham, p, 48)

    _, a, b = _both(T, ctx, lat, dtype, run)
    assert np.array_equal(a, b)
    if diag != 1:
        ref = orc.moments(lat, orc.random_state(lat.n, 9, 0), rescale=rho, num_moments=48)
        assert np.abs(a[0] - ref).max() <= (TOL64 if dtype == 0 else TOL32)


def test_table_with_given_states_and_ldos(T, ctx, orc):
    """The table under the per-site paths: LDOS sites and given initial states."""
    lat = graphene(80, 70, disorder_w=1.0, seed=24)
    sites = np.array([0, 17, 4000, lat.n - 1], dtype=np.int64)

    def run(ham):
        p, keep = T.make_params(9.0, 24, 1, block=1, seed=3, sites=sites)
        return T.tbpm_propagate_dos(ctx.handle, ham, p)

    _, a, b = _both(T, ctx, lat, 0, run)
    assert np.array_equal(a["ldos"], b["ldos"])
    assert np.array_equal(a["corr"], b["corr"])


def test_no_table_for_many_hopping_values(T, ctx):
    lat = graphene(96)
    rng = np.random.default_rng(2)
    off = lat.col != np.repeat(np.arange(lat.n), np.diff(lat.row_ptr))
    v = lat.val.copy()
    # a random hopping per bond, kept Hermitian: H_ij = conj(H_ji)
    rows = np.repeat(np.arange(lat.n), np.diff(lat.row_ptr))
    key = np.minimum(rows, lat.col).astype(np.int64) * lat.n + np.maximum(rows, lat.col)
    _, inv = np.unique(key, return_inverse=True)
    bond = -2.7 + 0.05 * rng.standard_normal(inv.max() + 1)
    v[off] = bond[inv[off]]
    ham = ctx.build(SimpleNamespace(n=lat.n, row_ptr=lat.row_ptr, col=lat.col, val=v), fmt=T.TBPM_FMT_PATCH)
    try:
        assert T.tbpm_ham_value_table(ham) == {"entries": 0, "per_row_diagonal": 0}
        assert T.tbpm_ham_info(ham)["format"] == T.TBPM_FMT_PATCH
    finally:
        T.tbpm_ham_destroy(ham)
