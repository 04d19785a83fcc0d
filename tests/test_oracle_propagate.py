"""Pins of the oracle's propagator and correlation function.

The oracle follows the Chebyshev recurrence step by step; these tests pin it
to results fixed by other means:
  * exact diagonalization on tiny lattices: C(t) = sum_n |<E_n|psi0>|^2 e^{-i E_n t};
  * one step against exp(-i H dt) psi0 built from the eigenvectors;
  * Bloch sums on clean periodic graphene of any size, with H(k) written here
    from the paper's graphene hopping list (independent of tb_inputs);
  * the square-lattice single-site return amplitude, a product of two 1-D
    ring sums, which tends to J_0(2|t| t)^2 before revivals;
  * unitarity, C(0) = 1, |C| <= 1, and the rescale check.
"""
import numpy as np
import pytest
from scipy import special

from tb_inputs import graphene, bilayer, square, honeycomb3, supercell, square_cell, state_from_sites


def _ed_corr(lat, psi0, t):
    e, v = np.linalg.eigh(lat.to_dense())
    a = np.abs(v.conj().T @ psi0) ** 2
    return np.exp(-1j * np.outer(t, e)) @ a


TINY = [
    ("graphene4_W1", lambda: graphene(4, disorder_w=1.0, seed=2), 9.0),
    ("graphene6_W1", lambda: graphene(6, disorder_w=1.0, seed=7), 9.0),
    ("bilayer4_W1", lambda: bilayer(4, disorder_w=1.0, seed=3), 9.0),
    ("honeycomb3_8_vac", lambda: honeycomb3(8, vacancy_p=0.05, seed=5), 10.0),
    ("square16_nnn", lambda: square(16), 4.5),
    ("graphene_3x5", lambda: graphene(3, 5), 9.0),
]


@pytest.mark.parametrize("name,make,rho", TINY, ids=[t[0] for t in TINY])
def test_exact_diagonalization(orc, name, make, rho):
    lat = make()
    nt = 256
    psi0 = orc.random_state(lat.n, 1, 0)
    res = orc.propagate(lat, psi0, rescale=rho, num_steps=nt)
    t = np.arange(nt + 1) * np.pi / rho
    ref = _ed_corr(lat, psi0, t)
    err = np.abs(res.corr - ref).max()
    assert err < 2e-12, err
    assert res.num_terms == 20


def test_exact_diagonalization_other_dt(orc):
    # a longer step (tau = 6) exercises more terms and the general dt argument
    lat = graphene(5, disorder_w=1.0, seed=9)
    psi0 = orc.random_state(lat.n, 3, 1)
    rho, dt, nt = 9.0, 6.0 / 9.0, 64
    res = orc.propagate(lat, psi0, rescale=rho, num_steps=nt, dt=dt)
    ref = _ed_corr(lat, psi0, np.arange(nt + 1) * dt)
    assert np.abs(res.corr - ref).max() < 1e-12
    assert res.num_terms > 20


def test_one_step_state(orc):
    lat = bilayer(3, disorder_w=1.0, seed=1)
    rho = 9.0
    psi0 = orc.random_state(lat.n, 4, 0)
    res = orc.propagate(lat, psi0, rescale=rho, num_steps=1, keep_final=True)
    e, v = np.linalg.eigh(lat.to_dense())
    exact = v @ (np.exp(-1j * e * np.pi / rho) * (v.conj().T @ psi0))
    # truncation error bound per step: sum_{m>=20} 2|J_m(pi)| ~ 7e-15
    assert np.linalg.norm(res.psi_final - exact) < 1.5e-14


def _bloch_corr_graphene(psi0, la, lb, t_hop, times):
    from bloch import corr_graphene
    return corr_graphene(psi0, la, lb, t_hop, times)


@pytest.mark.parametrize("la,lb", [(16, 16), (64, 64), (10, 24)])
def test_bloch_sum_clean_graphene(orc, la, lb):
    # 64 x 64 with rho = 9, 256 steps, seed 1 is the first (small) workload exactly
    lat = graphene(la, lb)
    psi0 = orc.random_state(lat.n, 1, 0)
    nt = 256
    res = orc.propagate(lat, psi0, rescale=9.0, num_steps=nt)
    ref = _bloch_corr_graphene(psi0, la, lb, -2.7, np.arange(nt + 1) * np.pi / 9.0)
    assert np.abs(res.corr - ref).max() < 1e-12


def test_graphene_spectrum_matches_dispersion():
    lat = graphene(6, 4)
    e = np.sort(np.linalg.eigvalsh(lat.to_dense()))
    ka, kb = np.meshgrid(2 * np.pi * np.arange(6) / 6, 2 * np.pi * np.arange(4) / 4, indexing="ij")
    ek = 2.7 * np.abs(1 + np.exp(1j * ka) + np.exp(1j * kb)).ravel()
    np.testing.assert_allclose(e, np.sort(np.concatenate([-ek, ek])), atol=1e-12)


@pytest.mark.parametrize("L", [32, 64])
def test_square_single_site_closed_form(orc, L):
    th = -1.0
    lat = supercell(square_cell(th, 0.0), L, L)
    rho, nt = 4.5, 60
    psi0 = state_from_sites(lat.n, [0])
    res = orc.propagate(lat, psi0, rescale=rho, num_steps=nt)
    t = np.arange(nt + 1) * np.pi / rho
    q = 2 * np.pi * np.arange(L) / L
    ring = np.exp(-2j * th * np.outer(t, np.cos(q))).mean(axis=1)
    assert np.abs(res.corr - ring ** 2).max() < 1e-13
    # before the first revival (t < L / (2|t|) roughly) the ring sum is J_0(2|t| t)
    early = t < 0.35 * L / (2 * abs(th))
    assert np.abs(res.corr[early] - special.jv(0, 2 * abs(th) * t[early]) ** 2).max() < 1e-12


def test_unitarity_and_special_values(orc):
    lat = graphene(12, disorder_w=1.0, seed=4)
    psi0 = orc.random_state(lat.n, 8, 0)
    res = orc.propagate(lat, psi0, rescale=9.0, num_steps=256)
    dev = np.abs(res.norms - 1)
    assert dev.max() < 1e-12
    # C(0) = sum_i |psi0_i|^2 = 1 up to the rounding of a length-N sum
    assert abs(res.corr[0] - 1) < lat.n * 2.3e-16 and res.corr[0].imag == 0
    assert np.all(np.abs(res.corr) <= 1 + 1e-12)


def test_site_correlation_consistency(orc):
    lat = honeycomb3(6, vacancy_p=0.03, seed=2)
    rho = 10.0
    psi0 = orc.random_state(lat.n, 9, 0)
    sites = [0, 5, lat.n - 1]
    res = orc.propagate(lat, psi0, rescale=rho, num_steps=8, sites=sites, keep_final=True)
    for s, i in enumerate(sites):
        assert abs(res.site_corr[s, -1] - np.conj(psi0[i]) * res.psi_final[i]) < 1e-18
        assert abs(res.site_corr[s, 0] - np.conj(psi0[i]) * psi0[i]) < 1e-18
    # a state localized on one site: the site correlation is the full correlation
    loc = state_from_sites(lat.n, [7])
    r2 = orc.propagate(lat, loc, rescale=rho, num_steps=8, sites=[7])
    np.testing.assert_allclose(r2.site_corr[0], r2.corr, rtol=0, atol=1e-16)


def test_ldos_estimator_is_unbiased(orc):
    # average of N conj(psi0_i) psi_i(t) over many random vectors -> <i|e^{-iHt}|i>
    lat = graphene(3, disorder_w=1.0, seed=6)
    rho, nt, R = 9.0, 6, 4000
    sites = [0, 5]
    _, _, _, ld = orc.corr_dos(lat, rescale=rho, num_steps=nt, num_vectors=R, seed=21, sites=sites)
    e, v = np.linalg.eigh(lat.to_dense())
    t = np.arange(nt + 1) * np.pi / rho
    for s, i in enumerate(sites):
        exact = np.exp(-1j * np.outer(t, e)) @ (np.abs(v[i]) ** 2)
        assert np.abs(ld[s] - exact).max() < 6 / np.sqrt(R)


def test_rescale_below_gershgorin_rejected(orc):
    lat = graphene(4)
    psi0 = orc.random_state(lat.n, 1, 0)
    with pytest.raises(ValueError):
        orc.propagate(lat, psi0, rescale=8.0, num_steps=4)
    assert abs(orc.gershgorin(lat) - 8.1) < 1e-12


def test_hermitian_check(orc):
    lat = graphene(4, disorder_w=1.0, seed=1)
    assert orc.is_hermitian(lat)
    bad = graphene(4)
    bad.val = bad.val.copy()
    bad.val[3] = bad.val[3] + 0.5j
    assert not orc.is_hermitian(bad)


def test_zero_steps(orc):
    lat = graphene(4)
    psi0 = orc.random_state(lat.n, 1, 0)
    res = orc.propagate(lat, psi0, rescale=9.0, num_steps=0)
    assert res.corr.shape == (1,) and abs(res.corr[0] - 1) < 1e-14


def test_bloch_sum_square_nnn(orc):
    """The square lattice's Bloch sum (NN t = -1, NNN t' = 0.1) against exact
    diagonalization and the oracle, on a rectangular lattice."""
    from bloch import corr_square
    from tb_inputs import square
    lat = square(12, 10)
    psi0 = orc.random_state(lat.n, 5, 0)
    times = np.arange(41) * np.pi / 4.5
    ref = corr_square(psi0, 12, 10, -1.0, 0.1, times)
    assert np.abs(ref - _ed_corr(lat, psi0, times)).max() < 1e-12
    res = orc.propagate(lat, psi0, rescale=4.5, num_steps=40)
    assert np.abs(res.corr - ref).max() < 1e-12
