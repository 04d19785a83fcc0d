"""Pins of the oracle's DOS transform.

d(E) = (1/2pi) int e^{iEt} C(t) dt, sampled on E_j = -rho + j rho/N_t,
j < 2 N_t, from C(t_k), t_k = k pi/rho, with C(-t) = conj(C(t)).
Pinned by the discrete sum rule sum_j d_j rho/N_t = Re C_0, by the closed form
for a single level on the grid (a Dirichlet kernel), and by physics: the
random-vector DOS agrees with the exact (trace) DOS of the same lattice.
"""
import numpy as np
import pytest

from tb_inputs import graphene


@pytest.mark.parametrize("window", [0, 1])
def test_sum_rule(orc, window):
    rng = np.random.default_rng(0)
    nt, rho = 64, 9.0
    c = rng.normal(size=nt + 1) + 1j * rng.normal(size=nt + 1)
    e, d = orc.dos(c, rho, window)
    assert e.size == 2 * nt and abs(e[0] + rho) < 1e-15 and abs(e[1] - e[0] - rho / nt) < 1e-14
    assert abs(d.sum() * rho / nt - c[0].real) < 1e-12


def test_single_level_closed_form(orc):
    nt, rho = 50, 9.0
    dt = np.pi / rho
    j0 = 37
    e0 = -rho + j0 * rho / nt
    c = np.exp(-1j * e0 * dt * np.arange(nt + 1))
    e, d = orc.dos(c, rho, window=0)
    # sum_{k=1}^{N} cos(k x) = sin(N x / 2) cos((N+1) x / 2) / sin(x / 2)
    x = (np.arange(2 * nt) - j0) * np.pi / nt
    with np.errstate(invalid="ignore", divide="ignore"):
        dk = np.sin(nt * x / 2) * np.cos((nt + 1) * x / 2) / np.sin(x / 2)
    dk[j0] = nt
    ref = dt / (2 * np.pi) * (1 + 2 * dk)
    np.testing.assert_allclose(d, ref, atol=1e-12)
    assert np.argmax(d) == j0


def test_window_suppresses_ringing(orc):
    nt, rho = 64, 9.0
    dt = np.pi / rho
    e0 = 1.234
    c = np.exp(-1j * e0 * dt * np.arange(nt + 1))
    _, d0 = orc.dos(c, rho, 0)
    e, d1 = orc.dos(c, rho, 1)
    far = np.abs(e - e0) > 2.0
    assert np.abs(d1[far]).max() < 0.05 * np.abs(d0[far]).max()
    assert abs(e[np.argmax(d1)] - e0) <= rho / nt


def test_random_vector_dos_matches_trace_dos(orc):
    # E[C(t)] = Tr e^{-iHt} / N, so the averaged TBPM DOS approaches the exact DOS
    lat = graphene(24, disorder_w=0.5, seed=3)
    rho, nt, R = 9.0, 128, 8
    mean, per, norms, _ = orc.corr_dos(lat, rescale=rho, num_steps=nt, num_vectors=R, seed=17)
    e_vals = np.linalg.eigvalsh(lat.to_dense())
    t = np.arange(nt + 1) * np.pi / rho
    c_exact = np.exp(-1j * np.outer(t, e_vals)).mean(axis=1)
    assert np.abs(mean - c_exact).max() < 5 / np.sqrt(lat.n * R)
    e, d = orc.dos(mean, rho)
    _, d_ex = orc.dos(c_exact, rho)
    # noise of C is ~1/sqrt(N R) per time point; through the transform the DOS
    # noise is about dt/pi * sqrt(sum_k w_k^2) / sqrt(N R)
    w = 0.5 * (1 + np.cos(np.pi * np.arange(1, nt + 1) / nt))
    sigma = np.pi / rho / np.pi * np.sqrt((w ** 2).sum()) / np.sqrt(lat.n * R)
    assert np.abs(d - d_ex).max() < 5 * sigma
    # van Hove peaks of graphene near +-|t| = 2.7 eV
    pos = (e > 1.5) & (e < 4.0)
    assert abs(e[pos][np.argmax(d_ex[pos])] - 2.7) < 0.3
