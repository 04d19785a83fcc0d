"""Host checks of the value-table planner (no GPU): the table a stored H
would hold, on lattices whose distinct hopping values are known from their
definitions -- graphene's one hopping t, the AB bilayer's t and gamma_1, the
3rd-neighbour honeycomb's three hoppings, Anderson disorder on the diagonal
(kept per row), complex64 rounding, and matrices the table cannot cover."""
import numpy as np
import pytest

from tb_inputs import graphene, bilayer, honeycomb3
from types import SimpleNamespace


@pytest.fixture(scope="module")
def T():
    from paper_2509_26309_amd import tbpm
    return tbpm


def plan(T, lat, dtype=0):
    return T.tbpm_value_table_plan(lat.n, lat.row_ptr, lat.col, lat.val, dtype)


def _distinct_bits(vals, dtype=0):
    """Distinct values bit for bit (numpy's own count): a conjugate pair of a
    real hopping differs in the sign of its zero imaginary part."""
    v = np.asarray(vals, dtype=np.complex128 if dtype == 0 else np.complex64)
    v = v[(v.view(np.float64 if dtype == 0 else np.float32) != 0).reshape(-1, 2).any(axis=1)
          | np.signbit(v.view(np.float64 if dtype == 0 else np.float32)).reshape(-1, 2).any(axis=1)]
    w = v.view(np.uint64 if dtype == 0 else np.uint32).reshape(-1, 2)
    return len(np.unique(w, axis=0))


def _offdiag(lat):
    return lat.col != np.repeat(np.arange(lat.n), np.diff(lat.row_ptr))


def test_clean_lattices_hold_their_hoppings(T):
    # +0 (ELL padding) is always entry 0; then the distinct hoppings: graphene
    # has one, the AB bilayer two, the 3rd-neighbour honeycomb three
    for lat, hoppings in ((graphene(8), 1), (bilayer(6), 2), (honeycomb3(9, vacancy_p=0.05, seed=3), 3)):
        off = _offdiag(lat)
        assert len(np.unique(lat.val[off])) == hoppings
        assert plan(T, lat) == {"entries": 1 + _distinct_bits(lat.val[off]), "per_row_diagonal": 0}


def test_anderson_disorder_goes_to_the_per_row_diagonal(T):
    for lat in (graphene(20, disorder_w=1.0, seed=2), bilayer(12, disorder_w=1.0, seed=3)):
        off = _offdiag(lat)
        assert plan(T, lat) == {"entries": 1 + _distinct_bits(lat.val[off]), "per_row_diagonal": 2}


def test_complex_onsite_values_are_kept_whole(T):
    # an on-site value with a nonzero imaginary part: the per-row diagonal keeps both parts
    lat = graphene(20, disorder_w=1.0, seed=2)
    rows = np.repeat(np.arange(lat.n), np.diff(lat.row_ptr))
    v = lat.val.copy()
    d = np.nonzero(lat.col == rows)[0]
    v[d[0]] += 1e-3j
    lat2 = SimpleNamespace(n=lat.n, row_ptr=lat.row_ptr, col=lat.col, val=v)
    assert plan(T, lat2)["per_row_diagonal"] == 1


def test_few_onsite_values_stay_in_the_table(T):
    # two sublattice potentials +-0.1: the diagonal fits the table
    lat = graphene(10)
    lat2 = _with_diagonal(lat, np.where(np.arange(lat.n) % 2 == 0, 0.1, -0.1))
    assert plan(T, lat2) == {"entries": 1 + _distinct_bits(lat.val[_offdiag(lat)]) + 2, "per_row_diagonal": 0}


def test_complex64_merges_values_equal_after_rounding(T):
    lat = graphene(6)
    v = lat.val.copy()
    # perturb half the hoppings below the complex64 resolution of -2.7
    idx = np.nonzero(_offdiag(lat))[0][::2]
    v[idx] = v[idx] * (1 + 1e-12)
    lat2 = SimpleNamespace(n=lat.n, row_ptr=lat.row_ptr, col=lat.col, val=v)
    base = _distinct_bits(lat.val[_offdiag(lat)])
    assert plan(T, lat2, 0)["entries"] == 1 + _distinct_bits(v[_offdiag(lat)]) > 1 + base
    assert plan(T, lat2, 1)["entries"] == 1 + _distinct_bits(v[_offdiag(lat)], 1) == 1 + base


def test_many_hopping_values_give_no_table(T):
    lat = graphene(12)
    rng = np.random.default_rng(1)
    v = lat.val.copy()
    off = lat.col != np.repeat(np.arange(lat.n), np.diff(lat.row_ptr))
    v[off] = -2.7 + 0.01 * rng.standard_normal(int(off.sum()))
    lat2 = SimpleNamespace(n=lat.n, row_ptr=lat.row_ptr, col=lat.col, val=v)
    assert plan(T, lat2) == {"entries": 0, "per_row_diagonal": 0}


def test_254_hopping_values_fit_255_do_not(T):
    n = 600
    for k, fits in ((254, True), (255, False)):
        rows = [[] for _ in range(n)]
        vals = {}
        for j in range(k):                       # hopping j between rows j and j + 1 (and its conjugate)
            a, b = j, j + 1
            rows[a].append(b)
            rows[b].append(a)
            vals[(a, b)] = vals[(b, a)] = -1.0 - j * 0.001
        rp = np.zeros(n + 1, dtype=np.int64)
        col = []
        val = []
        for i in range(n):
            for c in sorted(rows[i]):
                col.append(c)
                val.append(vals[(i, c)])
            rp[i + 1] = len(col)
        got = T.tbpm_value_table_plan(n, rp, np.array(col, dtype=np.int32), np.array(val, dtype=np.complex128))
        assert got["entries"] == (k + 1 if fits else 0)


def test_bad_arguments(T):
    lat = graphene(4)
    with pytest.raises(T.TBPMError):
        T.tbpm_value_table_plan(lat.n, lat.row_ptr, lat.col, lat.val, 7)


def _with_diagonal(lat, d):
    rp, col, val = lat.row_ptr, lat.col, lat.val
    n = lat.n
    new_rp = np.zeros(n + 1, dtype=np.int64)
    cols, vals = [], []
    for i in range(n):
        c = list(col[rp[i]:rp[i + 1]])
        v = list(val[rp[i]:rp[i + 1]])
        if i in c:
            v[c.index(i)] += d[i]
        else:
            c.append(i)
            v.append(d[i])
        order = np.argsort(c)
        cols.extend(np.array(c)[order])
        vals.extend(np.array(v)[order])
        new_rp[i + 1] = len(cols)
    return SimpleNamespace(n=n, row_ptr=new_rp, col=np.array(cols, dtype=np.int32),
                           val=np.array(vals, dtype=np.complex128))
