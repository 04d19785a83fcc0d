"""GPU parity of the time-dependent wave function (snapshots of psi(t_k)) and
of the quasi-eigenstates q(E) = sum_k w_k e^{i E t_k} psi(t_k), through the C
ABI, against the oracle's propagate_outputs on the same states.
Tolerances as for the propagator: complex128 path 1e-10, complex64 path 1e-5
(absolute, elementwise; |psi_i| ~ n^-1/2 and |q_i| <= sum_k w_k |psi_i(t_k)|)."""
import numpy as np
import pytest

from tb_inputs import graphene, square, state_from_sites

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


def _with_ham(T, ctx, lat, dtype, fmt, fn):
    ham = ctx.build(lat, dtype=dtype, fmt=fmt)
    try:
        return fn(ham), T.tbpm_ham_info(ham)
    finally:
        T.tbpm_ham_destroy(ham)


CASES = [("csr", lambda: graphene(13, 11, disorder_w=1.0, seed=5), 0),
         ("ell", lambda: graphene(13, 11, disorder_w=1.0, seed=5), 1),
         ("patch", lambda: graphene(192, disorder_w=1.0, seed=2), 2)]


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("name,make,fmt", CASES, ids=[c[0] for c in CASES])
def test_snapshots(T, ctx, orc, name, make, fmt, dtype):
    lat = make()
    nt, steps = 40, [0, 1, 5, 17, 40, 17]
    p, _ = T.make_params(9.0, nt, 1, seed=3, first_vector=2)
    out, info = _with_ham(T, ctx, lat, dtype, fmt, lambda h: T.tbpm_time_evolution(ctx.handle, h, p, steps))
    if name == "patch":
        assert info["format"] == T.TBPM_FMT_PATCH
    psi0 = orc.random_state(lat.n, 3, 2)
    snaps, _ = orc.propagate_outputs(lat, psi0, rescale=9.0, num_steps=nt, snap_steps=steps)
    assert np.abs(out["snapshots"] - snaps).max() <= TOL[dtype]
    corr = orc.propagate(lat, psi0, rescale=9.0, num_steps=nt).corr
    assert np.abs(out["corr"] - corr).max() <= TOL[dtype]


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("name,make,fmt", CASES, ids=[c[0] for c in CASES])
def test_quasi_eigenstates(T, ctx, orc, name, make, fmt, dtype):
    lat = make()
    nt = 64
    energies = np.linspace(-8.0, 8.0, 21)                  # two groups of at most 16 energies
    p, _ = T.make_params(9.0, nt, 1, seed=4)
    out, _ = _with_ham(T, ctx, lat, dtype, fmt, lambda h: T.tbpm_quasi_eigenstates(ctx.handle, h, p, energies))
    _, qe = orc.propagate_outputs(lat, orc.random_state(lat.n, 4, 0), rescale=9.0, num_steps=nt, energies=energies)
    assert np.abs(out["qe"] - qe).max() <= TOL[dtype] * 8


def test_given_state_snapshots_and_qe(T, ctx, orc):
    """A site-localised state on the square lattice (given as psi0)."""
    lat = square(20)
    psi0 = state_from_sites(lat.n, [37])
    nt = 30
    p, _ = T.make_params(4.5, nt, 1)
    out, _ = _with_ham(T, ctx, lat, 0, 1, lambda h: T.tbpm_time_evolution(ctx.handle, h, p, [0, 30], psi0=psi0))
    snaps, _ = orc.propagate_outputs(lat, psi0, rescale=4.5, num_steps=nt, snap_steps=[0, 30])
    assert np.array_equal(out["snapshots"][0], psi0)
    assert np.abs(out["snapshots"] - snaps).max() <= 1e-10
    out, _ = _with_ham(T, ctx, lat, 0, 1, lambda h: T.tbpm_quasi_eigenstates(ctx.handle, h, p, [0.0, -0.4],
                                                                             psi0=psi0))
    _, qe = orc.propagate_outputs(lat, psi0, rescale=4.5, num_steps=nt, energies=[0.0, -0.4])
    assert np.abs(out["qe"] - qe).max() <= 1e-10


def test_no_time_steps(T, ctx, orc):
    lat = graphene(6)
    p, _ = T.make_params(9.0, 0, 1, seed=8)
    out, _ = _with_ham(T, ctx, lat, 0, 0, lambda h: T.tbpm_quasi_eigenstates(ctx.handle, h, p, [1.0]))
    assert np.abs(out["qe"][0] - orc.random_state(lat.n, 8, 0)).max() <= 1e-15


def test_wft_qe_errors(T, ctx):
    lat = graphene(6)
    ham = ctx.build(lat)
    try:
        p, _ = T.make_params(9.0, 10, 2)
        with pytest.raises(T.TBPMError) as ei:
            T.tbpm_time_evolution(ctx.handle, ham, p, [1])
        assert ei.value.status == T.TBPM_ERR_ARG
        p, _ = T.make_params(9.0, 10, 1)
        with pytest.raises(T.TBPMError):
            T.tbpm_time_evolution(ctx.handle, ham, p, [11])
        with pytest.raises(T.TBPMError):
            T.tbpm_time_evolution(ctx.handle, ham, p, [])
        with pytest.raises(T.TBPMError):
            T.tbpm_quasi_eigenstates(ctx.handle, ham, p, [])
        with pytest.raises(T.TBPMError):
            T.tbpm_quasi_eigenstates(ctx.handle, ham, p, [np.nan])
        p, _ = T.make_params(5.0, 10, 1)
        with pytest.raises(T.TBPMError) as ei:
            T.tbpm_quasi_eigenstates(ctx.handle, ham, p, [0.0])
        assert ei.value.status == T.TBPM_ERR_RESCALE
    finally:
        T.tbpm_ham_destroy(ham)
