"""Pins of the oracle's random-phase states and Chebyshev coefficients.

Random states: the SplitMix64 output sequence is checked against the published
reference outputs (tests/golden), the counter form used for whole vectors
against the stream definition, and the phases against uniformity.
Coefficients: c_m = (2 - delta_m0)(-i)^m J_m(tau) are pinned by the
Jacobi-Anger identity sum_m c_m T_m(y) = exp(-i tau y), by Bessel sum rules
and by an independent Bessel routine (scipy), which the oracle does not use.
"""
import os

import numpy as np
import pytest
from scipy import special, stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_u64(name):
    vals = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                vals.append(int(line))
    return vals


def test_splitmix64_reference_sequence(orc):
    expected = _golden_u64("splitmix64_seed1234567.txt")
    got = [int(v) for v in orc.splitmix64_sequence(1234567, len(expected))]
    assert got == expected


def test_counter_form_matches_stream_definition(orc):
    n = 300
    for seed, r in [(1, 0), (1, 3), (2 ** 63 + 5, 2), (0, 0)]:
        psi = orc.random_state(n, seed, r)
        u_phase = np.mod(np.angle(psi) / (2 * np.pi), 1.0)
        for i in [0, 1, 2, 17, 150, n - 1]:
            u = orc.phase_u(seed, r, i)
            d = abs(u_phase[i] - u)
            assert min(d, 1 - d) < 1e-14, (seed, r, i)


def test_random_state_amplitude_and_norm(orc):
    for n in [1, 7, 1000, 65537]:
        psi = orc.random_state(n, 11, 2)
        np.testing.assert_allclose(np.abs(psi), 1 / np.sqrt(n), rtol=1e-15, atol=0)
        assert abs(np.vdot(psi, psi).real - 1) < 1e-13


def test_phases_uniform_and_streams_independent(orc):
    n = 200_000
    a = orc.random_state(n, 5, 0)
    b = orc.random_state(n, 5, 1)
    c = orc.random_state(n, 6, 0)
    for v in (a, b, c):
        u = np.mod(np.angle(v) / (2 * np.pi), 1.0)
        assert stats.kstest(u, "uniform").pvalue > 1e-4
    # <a|b> of independent random-phase states is O(1/sqrt(n))
    for x, y in [(a, b), (a, c), (b, c)]:
        assert abs(np.vdot(x, y)) < 6 / np.sqrt(n)
    assert not np.array_equal(a, orc.random_state(n, 5, 2))


def test_truncation_count_at_pi(orc):
    # tau = pi, eps = 1e-14: J_19(pi) = 3.9e-14 is kept, J_20(pi) = 3.1e-15 is not
    c = orc.coefficients(np.pi, 1e-14)
    assert c.size == 20
    assert abs(special.jv(19, np.pi)) >= 1e-14 > abs(special.jv(20, np.pi))


@pytest.mark.parametrize("tau,eps", [(np.pi, 1e-14), (5.0, 1e-12), (0.5, 1e-14), (30.0, 1e-13), (np.pi, 1e-6)])
def test_truncation_rule(orc, tau, eps):
    c = orc.coefficients(tau, eps)
    m = c.size
    assert m > tau
    assert abs(special.jv(m, tau)) < eps
    # every earlier index past tau is at or above eps
    for k in range(int(np.floor(tau)) + 1, m):
        assert abs(special.jv(k, tau)) >= eps


@pytest.mark.parametrize("tau,eps,tol", [(np.pi, 1e-14, 2e-14), (5.0, 1e-12, 3e-11), (30.0, 1e-13, 5e-12),
                                         (0.5, 1e-14, 3e-14)])
def test_jacobi_anger_identity(orc, tau, eps, tol):
    c = orc.coefficients(tau, eps)
    y = np.linspace(-1, 1, 401)
    m = np.arange(c.size)
    t = np.cos(np.outer(m, np.arccos(y)))          # T_m(y)
    series = c @ t
    np.testing.assert_array_less(np.abs(series - np.exp(-1j * tau * y)), tol)


def test_coefficients_match_independent_bessel(orc):
    for tau in [np.pi, 2.0, 7.5]:
        c = orc.coefficients(tau, 1e-14)
        m = np.arange(c.size)
        phase = (-1j) ** m
        scale = np.where(m == 0, 1.0, 2.0)
        ref = scale * phase * special.jv(m, tau)
        np.testing.assert_allclose(c, ref, rtol=0, atol=1e-15)
        # exact phase pattern: real for even m, imaginary for odd m
        assert np.all(c[0::2].imag == 0) and np.all(c[1::2].real == 0)


def test_bessel_sum_rules(orc):
    c = orc.coefficients(np.pi, 1e-16)
    j = np.abs(c) / np.where(np.arange(c.size) == 0, 1.0, 2.0)
    sgn = np.sign((c * (1j) ** np.arange(c.size)).real)   # recovers sign of J_m
    jm = sgn * j
    # J_0 + 2 sum_k J_2k = 1 ; J_0^2 + 2 sum_m J_m^2 = 1
    assert abs(jm[0] + 2 * jm[2::2].sum() - 1) < 1e-15
    assert abs(jm[0] ** 2 + 2 * (jm[1:] ** 2).sum() - 1) < 1e-15
