"""Checks of the synthetic lattice generators (sizes, symmetry, spectra)."""
import numpy as np
import pytest

from tb_inputs import graphene, bilayer, square, honeycomb3, sample_sites


def _dense_hermitian(lat):
    h = lat.to_dense()
    return np.abs(h - h.conj().T).max() == 0.0, h


def test_first_workload_sizes():
    lat = graphene(64)
    assert lat.n == 8192 and lat.nnz == 24576
    assert np.all(np.diff(lat.row_ptr) == 3)


def test_sorted_columns_and_range():
    for lat in [graphene(5, disorder_w=1.0, seed=1), bilayer(4), square(6), honeycomb3(7, vacancy_p=0.1, seed=3)]:
        assert lat.col.min() >= 0 and lat.col.max() < lat.n
        for i in range(lat.n):
            c = lat.col[lat.row_ptr[i]:lat.row_ptr[i + 1]]
            assert np.all(np.diff(c) > 0)


def test_counts_per_cell():
    assert graphene(8, disorder_w=1.0, seed=2).nnz == 8 * 8 * 2 * 4        # 3 hops + diagonal
    b = bilayer(8, disorder_w=1.0, seed=3)
    assert b.n == 8 * 8 * 4 and b.nnz == 8 * 8 * 18                          # 12 intra + 2 gamma1 + 4 diag
    assert square(8).nnz == 64 * 8
    assert honeycomb3(8).nnz == 128 * 12


@pytest.mark.parametrize("make", [lambda: graphene(5, disorder_w=1.0, seed=1), lambda: bilayer(4, disorder_w=1.0, seed=3),
                                  lambda: square(7), lambda: honeycomb3(6, vacancy_p=0.05, seed=2), lambda: graphene(2),
                                  lambda: graphene(1)])
def test_hermitian(make):
    ok, _ = _dense_hermitian(make())
    assert ok


def test_spectral_bounds():
    # clean graphene: [-3|t|, 3|t|]; square NN+NNN (t=-1, t'=0.1): [-3.6, 4.4]
    e = np.linalg.eigvalsh(graphene(6).to_dense())
    assert abs(e.max() - 8.1) < 1e-12 and abs(e.min() + 8.1) < 1e-12
    e = np.linalg.eigvalsh(square(8).to_dense())
    assert abs(e.min() + 3.6) < 1e-12 and e.max() <= 4.4 + 1e-12
    e = np.linalg.eigvalsh(honeycomb3(12).to_dense())
    assert e.min() > -9.85 and e.max() < 7.45


def test_disorder_range_and_seed():
    a = graphene(8, disorder_w=1.0, seed=2)
    b = graphene(8, disorder_w=1.0, seed=2)
    c = graphene(8, disorder_w=1.0, seed=3)
    assert np.array_equal(a.val, b.val) and not np.array_equal(a.val, c.val)
    assert a.onsite.min() >= -0.5 and a.onsite.max() <= 0.5


def test_vacancies():
    full = honeycomb3(20)
    vac = honeycomb3(20, vacancy_p=0.01, seed=5)
    assert vac.n < full.n and abs(vac.n / full.n - 0.99) < 0.01
    assert np.all(np.diff(vac.kept) > 0)
    assert np.diff(vac.row_ptr).max() == 12


def test_sample_sites():
    s = sample_sites(1000, 64, 55)
    assert s.size == 64 and np.all(np.diff(s) > 0) and s.max() < 1000


def test_operator_geometry():
    """Hop displacements are the neighbour distances; J = i[H, x] away from the
    periodic seam (positions unwrapped); rho_q is unitary and diagonal."""
    from tb_inputs import (hop_displacements, current_operator, density_operator, positions, area_per_orbital,
                           honeycomb3)
    lat = graphene(6)
    d = np.linalg.norm(hop_displacements(lat), axis=1)
    np.testing.assert_allclose(d, 0.246 / np.sqrt(3.0), rtol=1e-12)
    lat3 = honeycomb3(7)
    d3 = np.unique(np.round(np.linalg.norm(hop_displacements(lat3), axis=1), 6))
    np.testing.assert_allclose(d3, [0.246 / np.sqrt(3.0), 0.246, 2 * 0.246 / np.sqrt(3.0)], rtol=1e-5)
    lat = graphene(7, disorder_w=1.0, seed=1)
    J = current_operator(lat, (0.6, 0.8)).to_dense()
    np.testing.assert_allclose(J, J.conj().T, atol=1e-15)
    H = lat.to_dense()
    r = positions(lat) @ np.array([0.6, 0.8])
    comm = 1j * (H * r[None, :] - r[:, None] * H)
    ca = (np.arange(lat.n) // 2) // 7
    cb = (np.arange(lat.n) // 2) % 7
    interior = (np.abs(ca[:, None] - ca[None, :]) <= 1) & (np.abs(cb[:, None] - cb[None, :]) <= 1)
    np.testing.assert_allclose(J[interior], comm[interior], atol=1e-12)
    rho = density_operator(lat, (1.0, -2.0))
    assert np.array_equal(rho.col, np.arange(lat.n)) and np.allclose(np.abs(rho.val), 1.0)
    assert abs(area_per_orbital(graphene(5)) - 0.246 ** 2 * np.sqrt(3.0) / 4.0) < 1e-15
