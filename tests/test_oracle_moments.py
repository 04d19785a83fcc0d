"""Pins of the oracle's Chebyshev-moment route (kernel polynomial method).

mu_m = <psi0|T_m(H/rho)|psi0> is computed by the oracle with the plain
Chebyshev recurrence and one inner product per moment; these tests fix it by
other means:
  * the spectral definition: mu_m = sum_n |<E_n|psi0>|^2 T_m(E_n/rho), with
    T_m(x) = cos(m arccos x), from exact diagonalization;
  * a Bloch sum for one site of the clean square lattice,
    mu_m = L^-2 sum_q T_m(2 t (cos q1 + cos q2) / rho);
  * C(t_k) rebuilt from the moments against exact diagonalization and against
    the step-by-step propagator;
  * the Jackson-damped DOS: Gauss-Chebyshev quadrature of the DOS returns
    mu_0 (sum rule), a single level gives a non-negative peak whose mean is
    x0 cos(pi/(N+1)) (the first Jackson factor) and whose width is the
    published resolution of about pi/N.
"""
import numpy as np
import pytest
from scipy import special

from tb_inputs import graphene, bilayer, honeycomb3, supercell, square_cell, state_from_sites

TINY = [
    ("graphene5_W1", lambda: graphene(5, disorder_w=1.0, seed=3), 9.0),
    ("bilayer3_W1", lambda: bilayer(3, disorder_w=1.0, seed=4), 9.0),
    ("honeycomb3_8_vac", lambda: honeycomb3(8, vacancy_p=0.05, seed=5), 10.0),
]


def _spectral_moments(lat, psi0, rho, num):
    e, v = np.linalg.eigh(lat.to_dense())
    a = np.abs(v.conj().T @ psi0) ** 2
    th = np.arccos(np.clip(e / rho, -1.0, 1.0))
    return np.array([np.sum(a * np.cos(m * th)) for m in range(num)]), e, a


@pytest.mark.parametrize("name,make,rho", TINY, ids=[t[0] for t in TINY])
def test_moments_spectral_definition(orc, name, make, rho):
    lat = make()
    psi0 = orc.random_state(lat.n, 11, 2)
    mu = orc.moments(lat, psi0, rescale=rho, num_moments=400)
    ref, _, _ = _spectral_moments(lat, psi0, rho, 400)
    # both sides carry rounding that grows like m * 1e-16: the recurrence's, and
    # m times the eigenvalue error inside cos(m arccos x)
    tol = 5e-15 + 4e-16 * np.arange(400)
    assert np.all(np.abs(mu - ref) < tol)
    assert abs(mu[0] - 1.0) < lat.n * 2.3e-16
    assert np.abs(mu).max() <= 1.0 + 1e-14


def test_moments_square_single_site_bloch_sum(orc):
    L, th, rho = 24, -1.0, 4.5
    lat = supercell(square_cell(th, 0.0), L, L)
    mu = orc.moments(lat, state_from_sites(lat.n, [0]), rescale=rho, num_moments=300)
    q = 2 * np.pi * np.arange(L) / L
    x = (2 * th * (np.cos(q)[:, None] + np.cos(q)[None, :]) / rho).ravel()
    ref = np.array([np.mean(np.cos(m * np.arccos(x))) for m in range(300)])
    assert np.abs(mu - ref).max() < 1e-13
    # odd moments of a bipartite lattice's site vanish
    assert np.abs(mu[1::2]).max() < 1e-14


def _moments_needed(nt, eps=1e-14):
    x = nt * np.pi
    m = int(np.ceil(x))
    while abs(special.jv(m, x)) >= eps:
        m += 1
    return m + 1


@pytest.mark.parametrize("name,make,rho", TINY, ids=[t[0] for t in TINY])
def test_corr_from_moments_exact_diagonalization(orc, name, make, rho):
    lat = make()
    psi0 = orc.random_state(lat.n, 5, 0)
    nt = 48
    mu = orc.moments(lat, psi0, rescale=rho, num_moments=_moments_needed(nt))
    corr = orc.corr_from_moments(mu, nt)
    t = np.arange(nt + 1) * np.pi / rho
    _, e, a = _spectral_moments(lat, psi0, rho, 1)
    ref = np.exp(-1j * np.outer(t, e)) @ a
    assert np.abs(corr - ref).max() < 1e-12


def test_corr_from_moments_agrees_with_propagator(orc):
    lat = graphene(10, disorder_w=1.0, seed=8)
    psi0 = orc.random_state(lat.n, 2, 1)
    nt = 128
    mu = orc.moments(lat, psi0, rescale=9.0, num_moments=_moments_needed(nt))
    corr = orc.corr_from_moments(mu, nt)
    res = orc.propagate(lat, psi0, rescale=9.0, num_steps=nt)
    assert np.abs(corr - res.corr).max() < 1e-12


def test_corr_from_too_few_moments_is_wrong(orc):
    # the truncation matters: half the moments miss the late times
    lat = graphene(6, disorder_w=1.0, seed=1)
    psi0 = orc.random_state(lat.n, 2, 0)
    nt = 40
    mu = orc.moments(lat, psi0, rescale=9.0, num_moments=_moments_needed(nt))
    good = orc.corr_from_moments(mu, nt)
    bad = orc.corr_from_moments(mu[: len(mu) // 2], nt)
    assert np.abs(good[: nt // 4] - bad[: nt // 4]).max() < 1e-12
    assert np.abs(good[-1] - bad[-1]) > 1e-3


def _quadrature(e, d, rho):
    # Gauss-Chebyshev: int f = (pi rho / K) sum_j f(E_j) sqrt(1 - x_j^2) at the nodes
    x = e / rho
    return np.pi * rho / e.size * d * np.sqrt(1.0 - x * x)


def test_kpm_dos_sum_rule(orc):
    lat = graphene(8, disorder_w=1.0, seed=2)
    psi0 = orc.random_state(lat.n, 4, 0)
    mu = orc.moments(lat, psi0, rescale=9.0, num_moments=256)
    e, d = orc.kpm_dos(mu, 9.0, 512)
    assert np.all(np.diff(e) > 0) and e[0] > -9.0 and e[-1] < 9.0
    assert abs(_quadrature(e, d, 9.0).sum() - mu[0].real) < 1e-13


@pytest.mark.parametrize("x0", [0.0, 0.3, -0.55])
def test_kpm_dos_single_level(orc, x0):
    n_mom, rho, k = 128, 2.0, 1024
    mu = np.cos(np.arange(n_mom) * np.arccos(x0)).astype(np.complex128)   # T_m(x0)
    e, d = orc.kpm_dos(mu, rho, k)
    w = _quadrature(e, d, rho)
    assert d.min() > -1e-12                       # the Jackson kernel is positive
    assert abs(w.sum() - 1.0) < 1e-13
    mean = (w * e / rho).sum()
    assert abs(mean - x0 * np.cos(np.pi / (n_mom + 1))) < 1e-13
    peak = e[np.argmax(d)] / rho
    assert abs(peak - x0) < 3.0 / n_mom
    if x0 == 0.0:
        var = (w * (e / rho) ** 2).sum()
        assert abs(var / (np.pi / n_mom) ** 2 - 1.0) < 0.05


def test_kpm_dos_graphene_van_hove(orc):
    # clean graphene, many vectors' worth of moments from one large lattice:
    # the DOS peaks at the van Hove energies +-|t| = +-2.7 eV
    lat = graphene(48)
    psi0 = orc.random_state(lat.n, 9, 0)
    mu = orc.moments(lat, psi0, rescale=9.0, num_moments=512)
    e, d = orc.kpm_dos(mu, 9.0, 2048)
    for sign in (-1, 1):
        sel = (sign * e > 1.5) & (sign * e < 4.0)
        assert abs(abs(e[sel][np.argmax(d[sel])]) - 2.7) < 0.1
