"""Pins of the oracle's response functions (Kubo formula by propagation):
  * the Fermi series sum_m a_m T_m(x) against f(rho x) itself;
  * corr(t) = <e^{-iHt} f(H) phi| A |e^{-iHt} (1 - f(H)) B phi> against exact
    diagonalization with the exact Fermi function, for current operators
    (AC conductivity) and density operators (dynamic polarization);
  * the limits mu far above / below the spectrum (f = 1 / f = 0: corr = 0);
  * the conductivity and polarization transforms of a two-level correlation
    against a numerical integral of the same windowed integrand (the sum over
    t_k is its rectangle rule, accurate to O(dt^4) here);
  * the universal optical conductivity of graphene, e^2 / (8 hbar) per spinless
    orbital channel, for hbar w between about 0.8 and 2 eV (statistical check).
Operators come from tb_inputs (J = i[H, x], rho_q = exp(i q.r)).
"""
import numpy as np
import pytest
from scipy import integrate

from tb_inputs import graphene, bilayer, current_operator, density_operator, area_per_orbital


@pytest.mark.parametrize("mu,kT", [(0.0, 0.05), (0.7, 0.2), (-2.0, 0.5)])
def test_fermi_series(orc, mu, kT):
    rho = 9.0
    a = orc.fermi_coefficients(rho, mu, kT)
    x = np.linspace(-1.0, 1.0, 3001)
    approx = np.cos(np.outer(np.arccos(x), np.arange(a.size))) @ a
    exact = 0.5 * (1.0 - np.tanh((rho * x - mu) / (2.0 * kT)))
    assert np.abs(approx - exact).max() < 1e-12
    assert abs(a[-1]) >= 1e-14 and a.size < 4 * rho / kT * 4


def _ed_corr(lat, phi, A, B, rho, nt, mu, kT):
    e, v = np.linalg.eigh(lat.to_dense())
    f = 0.5 * (1.0 - np.tanh((e - mu) / (2.0 * kT)))
    a0 = v.conj().T @ phi
    b0 = v.conj().T @ (B.to_dense() @ phi)
    Ad = A.to_dense()
    out = []
    for k in range(nt + 1):
        ph = np.exp(-1j * e * k * np.pi / rho)
        phi2 = v @ (ph * f * a0)
        phi1 = v @ (ph * (1.0 - f) * b0)
        out.append(np.vdot(phi2, Ad @ phi1))
    return np.array(out)


@pytest.mark.parametrize("kind", ["current_xx", "current_xy", "density"])
def test_response_corr_exact_diagonalization(orc, kind):
    lat = graphene(5, disorder_w=1.0, seed=3)
    if kind == "density":
        q = (2.0, 1.0)
        A, B = density_operator(lat, q), density_operator(lat, (-q[0], -q[1]))
    else:
        A = current_operator(lat, (1.0, 0.0))
        B = current_operator(lat, (1.0, 0.0) if kind == "current_xx" else (0.0, 1.0))
    phi = orc.random_state(lat.n, 5, 1)
    nt, rho, mu, kT = 30, 9.0, 0.4, 0.15
    got = orc.response_corr(lat, phi, A, B, rescale=rho, num_steps=nt, mu=mu, kT=kT)
    ref = _ed_corr(lat, phi, A, B, rho, nt, mu, kT)
    assert np.abs(got - ref).max() < 1e-11


def test_response_limits(orc):
    lat = bilayer(3, disorder_w=1.0, seed=2)
    J = current_operator(lat)
    phi = orc.random_state(lat.n, 1, 0)
    for mu in (60.0, -60.0):
        c = orc.response_corr(lat, phi, J, J, rescale=9.0, num_steps=8, mu=mu, kT=0.5)
        assert np.abs(c).max() < 1e-12


def test_conductivity_transform_two_level(orc):
    rho, nt, kT, om, delta, amp = 9.0, 200, 0.3, 0.02, 1.7, 0.8
    dt = np.pi / rho
    T = nt * dt
    t = np.arange(nt + 1) * dt
    corr = amp * np.exp(-1j * delta * t)
    w = np.array([0.5, 1.7, 3.0])
    got = orc.ac_conductivity(corr, rho, kT, om, w)
    for j, wj in enumerate(w):
        f = lambda s: 0.5 * (1 + np.cos(np.pi * s / T)) * np.sin(wj * s) * 2 * (-amp * np.sin(delta * s))
        val, _ = integrate.quad(f, 0.0, T, limit=800)
        pref = (np.exp(-wj / kT) - 1.0) / (wj * om)
        ref = pref * val
        # the sum over t_k is the rectangle rule of an integrand vanishing with its
        # slope at both ends: error O(dt^4), far below the scale of any mistake
        assert abs(got[j] - ref) < 1e-4 * abs(pref) * 2 * amp * T
    pol = orc.dyn_polarization(corr, rho, om, w)
    for j, wj in enumerate(w):
        g = lambda s, part: 0.5 * (1 + np.cos(np.pi * s / T)) * part(np.exp(1j * wj * s)) * (-amp * np.sin(delta * s))
        re, _ = integrate.quad(lambda s: g(s, np.real), 0.0, T, limit=800)
        im, _ = integrate.quad(lambda s: g(s, np.imag), 0.0, T, limit=800)
        # here the real integrand has slope -amp*delta at t = 0: the sum is the
        # trapezoid rule, integral + dt^2/12 (g'(T) - g'(0)) + O(dt^4)
        h = 1e-6
        slope = lambda s, part: (g(s + h, part) - g(s - h, part)) / (2 * h)
        re += dt * dt / 12.0 * (slope(T, np.real) - slope(0.0, np.real))
        im += dt * dt / 12.0 * (slope(T, np.imag) - slope(0.0, np.imag))
        ref = -2.0 / om * (re + 1j * im)
        assert abs(pol[j] - ref) < 1e-4 * 2.0 / om * amp * T


def test_graphene_universal_conductivity(orc):
    lat = graphene(256)
    J = current_operator(lat, (1.0, 0.0))
    phi = orc.random_state(lat.n, 3, 0)
    kT = 0.1
    corr = orc.response_corr(lat, phi, J, J, rescale=9.0, num_steps=128, mu=0.0, kT=kT)
    w = np.linspace(0.8, 2.0, 7)
    s = orc.ac_conductivity(corr, 9.0, kT, area_per_orbital(lat), w)
    assert abs(s.mean() - 0.125) < 0.02
    assert np.all((s > 0.08) & (s < 0.17))
