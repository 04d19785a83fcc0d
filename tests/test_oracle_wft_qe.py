"""Pins of the oracle's time-dependent wave function (snapshots of psi(t_k))
and quasi-eigenstates q(E) = sum_{k=0}^{N_t} w_k e^{i E t_k} psi(t_k) (Hann
weights w_k, t_k = k pi / rho):
  * exact diagonalization: psi(t_k) = sum_n e^{-i E_n t_k} <n|psi0> |n>, and
    q(E) = sum_n <n|psi0> |n> F(E - E_n), F(w) = sum_k w_k e^{i w t_k};
  * psi(t_0) = psi0 exactly, the last snapshot equals the propagator's final
    state bit for bit, and with no time steps q(E) = psi0;
  * discrete orthogonality: over the 2 N_t energies E_j = -rho + j rho / N_t,
    sum_j q(E_j) = 2 N_t psi0 (only the k = 0 term survives).
"""
import numpy as np
import pytest

from tb_inputs import graphene, bilayer, honeycomb3


def _ed(lat):
    e, v = np.linalg.eigh(lat.to_dense())
    return e, v


@pytest.mark.parametrize("make,rho", [(lambda: graphene(5, disorder_w=1.0, seed=3), 9.0),
                                      (lambda: honeycomb3(6, vacancy_p=0.05, seed=5), 10.0)])
def test_snapshots_exact_diagonalization(orc, make, rho):
    lat = make()
    psi0 = orc.random_state(lat.n, 4, 1)
    steps = [0, 1, 7, 40, 64]
    snaps, _ = orc.propagate_outputs(lat, psi0, rescale=rho, num_steps=64, snap_steps=steps)
    e, v = _ed(lat)
    a = v.conj().T @ psi0
    for s, k in enumerate(steps):
        ref = v @ (np.exp(-1j * e * k * np.pi / rho) * a)
        assert np.abs(snaps[s] - ref).max() < 1e-12
    assert np.array_equal(snaps[0], psi0)
    fin = orc.propagate(lat, psi0, rescale=rho, num_steps=64, keep_final=True).psi_final
    assert np.array_equal(snaps[-1], fin)


@pytest.mark.parametrize("nt", [1, 16, 100])
def test_quasi_eigenstates_exact_diagonalization(orc, nt):
    lat = bilayer(3, disorder_w=1.0, seed=2)
    rho = 9.0
    psi0 = orc.random_state(lat.n, 6, 0)
    energies = [-2.7, -0.4, 0.0, 1.3, 8.5]
    _, qe = orc.propagate_outputs(lat, psi0, rescale=rho, num_steps=nt, energies=energies)
    e, v = _ed(lat)
    a = v.conj().T @ psi0
    t = np.arange(nt + 1) * np.pi / rho
    w = 0.5 * (1.0 + np.cos(np.pi * np.arange(nt + 1) / nt))
    for j, E in enumerate(energies):
        f = (w[None, :] * np.exp(1j * np.outer(E - e, t))).sum(axis=1)
        ref = v @ (a * f)
        assert np.abs(qe[j] - ref).max() < 1e-11 * max(1.0, nt / 10)


def test_quasi_eigenstates_no_steps_and_orthogonality(orc):
    lat = graphene(4, disorder_w=1.0, seed=1)
    rho = 9.0
    psi0 = orc.random_state(lat.n, 2, 0)
    _, qe0 = orc.propagate_outputs(lat, psi0, rescale=rho, num_steps=0, energies=[0.3, -5.0])
    assert np.array_equal(qe0[0], psi0) and np.array_equal(qe0[1], psi0)
    nt = 24
    grid = -rho + np.arange(2 * nt) * rho / nt
    _, qe = orc.propagate_outputs(lat, psi0, rescale=rho, num_steps=nt, energies=grid)
    assert np.abs(qe.sum(axis=0) - 2 * nt * psi0).max() < 1e-12


def test_outputs_argument_errors(orc):
    lat = graphene(3)
    psi0 = orc.random_state(lat.n, 1, 0)
    with pytest.raises(RuntimeError):
        orc.propagate_outputs(lat, psi0, rescale=9.0, num_steps=4, snap_steps=[5])
    with pytest.raises(ValueError):
        orc.propagate_outputs(lat, psi0, rescale=3.0, num_steps=4, snap_steps=[1])
