"""Host-only functions of the moment route (no GPU): the number of moments a
time range needs, C(t) from moments, and the Jackson-kernel DOS, against the
oracle and scipy."""
import numpy as np
import pytest
from scipy import special

from tb_inputs import graphene, bilayer


@pytest.fixture(scope="module")
def T():
    from paper_2509_26309_amd import tbpm
    return tbpm


@pytest.mark.parametrize("nt", [1, 7, 48, 256, 1024, 4096])
def test_moments_needed_truncation(T, nt):
    m = T.tbpm_moments_needed(nt)
    x = nt * np.pi
    assert m > x and abs(special.jv(m, x)) < 1e-14
    assert all(abs(special.jv(k, x)) >= 1e-14 for k in range(int(x) + 1, m))


def test_moments_needed_edges(T):
    assert T.tbpm_moments_needed(0) == 1
    assert T.tbpm_moments_needed(1) == 20          # one step of the propagator's series
    with pytest.raises(Exception):
        T.tbpm_moments_needed(-1)
    with pytest.raises(Exception):
        T.tbpm_moments_needed(10, 0.0)


@pytest.mark.parametrize("nt", [1, 64, 300])
def test_corr_from_moments_matches_oracle(T, orc, nt):
    lat = bilayer(4, disorder_w=1.0, seed=3)
    psi0 = orc.random_state(lat.n, 8, 0)
    nm = T.tbpm_moments_needed(nt)
    mu = orc.moments(lat, psi0, rescale=9.0, num_moments=nm)
    got = T.tbpm_corr_from_moments(mu, nt)
    ref = orc.corr_from_moments(mu, nt)
    assert np.abs(got - ref).max() < 1e-13
    # and the propagator of the same state
    res = orc.propagate(lat, psi0, rescale=9.0, num_steps=nt)
    assert np.abs(got - res.corr).max() < 1e-12


def test_corr_from_moments_single_moment(T):
    got = T.tbpm_corr_from_moments(np.array([1.0 + 0j]), 5)
    x = np.arange(6) * np.pi
    np.testing.assert_allclose(got.real, special.jv(0, x), atol=1e-15)
    assert np.abs(got.imag).max() == 0.0


@pytest.mark.parametrize("num,k", [(64, 200), (255, 1024), (1000, 2048)])
def test_kpm_dos_matches_oracle(T, orc, num, k):
    lat = graphene(10, disorder_w=1.0, seed=6)
    mu = orc.moments(lat, orc.random_state(lat.n, 3, 0), rescale=9.0, num_moments=num)
    e, d = T.tbpm_kpm_dos(mu, 9.0, k)
    e2, d2 = orc.kpm_dos(mu, 9.0, k)
    assert np.abs(e - e2).max() < 1e-14
    assert np.abs(d - d2).max() < 1e-12


def test_host_argument_errors(T):
    with pytest.raises(Exception):
        T.tbpm_kpm_dos(np.ones(4, np.complex128), -1.0, 10)
    with pytest.raises(Exception):
        T.tbpm_kpm_dos(np.ones(4, np.complex128), 1.0, 0)
    with pytest.raises(Exception):
        T.tbpm_corr_from_moments(np.ones(4, np.complex128), -1)
