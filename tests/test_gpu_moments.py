"""GPU parity of the Chebyshev-moment route (through the C ABI) against the oracle.

The GPU forms mu_m with the doubling identities (two inner products per
product with H); the oracle takes one inner product per moment with the plain
recurrence.  Tolerances as for the propagator:
  FP64 (complex128 H and vectors):  max_m |mu_gpu - mu_oracle| <= 1e-10
  FP32 (complex64 H and vectors):   max_m |mu_gpu - mu_oracle| <= 1e-5
The FP64 bound covers summation order (~1e-16 sqrt(N) per inner product, times
two for the doubling); the FP32 bound covers the rounding of psi0 and of every
stored p_m to complex64 (~6e-8 relative each), growing at most linearly in m.
"""
import numpy as np
import pytest

from tb_inputs import graphene, bilayer, honeycomb3, square, sample_sites

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5


@pytest.fixture(scope="module")
def T():
    from paper_2509_26309_amd import tbpm
    return tbpm


@pytest.fixture(scope="module")
def ctx(T):
    c = T.Context(0)
    yield c
    c.close()


def _gpu(T, ctx, lat, *, rho, num, R=1, seed=1, dtype=0, fmt=2, block=0, lpr=0, first=0, flags=0):
    ham = ctx.build(lat, dtype=dtype, fmt=fmt, flags=flags)
    try:
        p, _ = T.make_params(rho, 0, R, block=block, seed=seed, lanes_per_row=lpr, first_vector=first)
        mu = T.tbpm_chebyshev_moments(ctx.handle, ham, p, num)
        info = T.tbpm_ham_info(ham)
    finally:
        T.tbpm_ham_destroy(ham)
    return mu, info


def _oracle(orc, lat, *, rho, num, R=1, seed=1, first=0):
    return np.stack([orc.moments(lat, orc.random_state(lat.n, seed, first + r), rescale=rho, num_moments=num)
                     for r in range(R)])


@pytest.mark.parametrize("num", [1, 2, 3, 4, 129, 301])
@pytest.mark.parametrize("fmt", [0, 1])
def test_moments_fp64(T, ctx, orc, fmt, num):
    """286 rows (a ragged tail in every tiling); 301 moments span three reduction chunks."""
    lat = graphene(13, 11, disorder_w=1.0, seed=5)
    mu, info = _gpu(T, ctx, lat, rho=9.0, num=num, fmt=fmt)
    ref = _oracle(orc, lat, rho=9.0, num=num)
    assert info["format"] == fmt
    assert mu.shape == (1, num)
    assert np.abs(mu - ref).max() <= TOL64


@pytest.mark.parametrize("lpr", [1, 2, 4, 8, 16])
def test_moments_csr_lanes(T, ctx, orc, lpr):
    lat = square(12)                                      # 8 entries per row
    mu, _ = _gpu(T, ctx, lat, rho=4.5, num=160, fmt=0, lpr=lpr, seed=4)
    ref = _oracle(orc, lat, rho=4.5, num=160, seed=4)
    assert np.abs(mu - ref).max() <= TOL64


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("block", [1, 2, 4, 8, 16, 32, 64])
def test_moments_blocks(T, ctx, orc, block, fmt, dtype):
    lat = graphene(9, 7, disorder_w=1.0, seed=8)
    R = block + 3 if block < 64 else 64                   # ragged: blocks of `block`, then 2, 1
    mu, _ = _gpu(T, ctx, lat, rho=9.0, num=100, R=R, block=block, seed=77, fmt=fmt, dtype=dtype, first=2)
    ref = _oracle(orc, lat, rho=9.0, num=100, R=R, seed=77, first=2)
    tol = TOL64 if dtype == 0 else TOL32
    assert np.abs(mu - ref).max() <= tol


def test_moments_ell_width12_block8_fp32(T, ctx, orc):
    """Third-neighbour honeycomb with vacancies: complex64 ELL, 8-vector blocks."""
    lat = honeycomb3(40, vacancy_p=0.01, seed=5)
    mu, info = _gpu(T, ctx, lat, rho=10.0, num=512, R=8, block=8, seed=5, dtype=1, fmt=1)
    ref = _oracle(orc, lat, rho=10.0, num=512, R=8, seed=5)
    assert info["format"] == 1
    assert np.abs(mu - ref).max() <= TOL32


@pytest.fixture(scope="module")
def lat192():
    return graphene(192, disorder_w=1.0, seed=2)          # 73,728 rows: AUTO picks patches


@pytest.fixture(scope="module")
def ref192(orc, lat192):
    return _oracle(orc, lat192, rho=9.0, num=203, seed=3)


@pytest.mark.parametrize("large", [False, True])
@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("num", [4, 5, 6, 200, 201, 203])
def test_moments_patch_format(T, ctx, lat192, ref192, num, dtype, large):
    """Patch-reordered ELL (rows renumbered), one vector: product 0 alone, then fused
    pairs of products, then one single product when their number is odd."""
    flags = T.TBPM_BUILD_LARGE_PATCHES if large else 0
    mu, info = _gpu(T, ctx, lat192, rho=9.0, num=num, seed=3, dtype=dtype, flags=flags)
    assert info["format"] == T.TBPM_FMT_PATCH
    tol = TOL64 if dtype == 0 else TOL32
    assert np.abs(mu[0] - ref192[0, :num]).max() <= tol


@pytest.mark.parametrize("num", [200, 203])
def test_moments_patch_pairs_profiled(T, ctx, lat192, ref192, num):
    T.tbpm_ctx_set_profiling(ctx.handle, True)
    try:
        mu, _ = _gpu(T, ctx, lat192, rho=9.0, num=num, seed=3)
        counts = [T.tbpm_ctx_kernel_time(ctx.handle, k)[1] for k in range(3)]
    finally:
        T.tbpm_ctx_set_profiling(ctx.handle, False)
    kmax = (num + 1) // 2
    assert counts == [1, (kmax - 1) // 2, (kmax - 1) % 2]
    assert np.abs(mu[0] - ref192[0, :num]).max() <= TOL64


def test_moments_patch_block4(T, ctx, orc, lat192, ref192):
    """Blocks wider than one vector on the patch format take the single-product kernels."""
    mu, _ = _gpu(T, ctx, lat192, rho=9.0, num=64, R=4, block=4, seed=3)
    ref = np.concatenate([ref192[:, :64], _oracle(orc, lat192, rho=9.0, num=64, R=3, seed=3, first=1)])
    assert np.abs(mu - ref).max() <= TOL64


def test_corr_from_gpu_moments_matches_propagators(T, ctx, orc):
    """C(t_k) from GPU moments against the oracle's step-by-step propagator and the GPU propagator."""
    lat = graphene(32, disorder_w=1.0, seed=4)
    nt = 256
    num = T.tbpm_moments_needed(nt)
    mu, _ = _gpu(T, ctx, lat, rho=9.0, num=num, seed=6)
    corr = T.tbpm_corr_from_moments(mu[0], nt)
    res = orc.propagate(lat, orc.random_state(lat.n, 6, 0), rescale=9.0, num_steps=nt)
    assert np.abs(corr - res.corr).max() <= TOL64
    ham = ctx.build(lat)
    try:
        p, _ = T.make_params(9.0, nt, 1, seed=6)
        prop = T.tbpm_propagate_dos(ctx.handle, ham, p)["corr"][0]
    finally:
        T.tbpm_ham_destroy(ham)
    assert np.abs(corr - prop).max() <= TOL64


def test_moments_exact_diagonalization(T, ctx):
    lat = bilayer(4, disorder_w=1.0, seed=3)
    mu, _ = _gpu(T, ctx, lat, rho=9.0, num=300, seed=1)
    from oracle import random_state
    psi0 = random_state(lat.n, 1, 0)
    e, v = np.linalg.eigh(lat.to_dense())
    a = np.abs(v.conj().T @ psi0) ** 2
    th = np.arccos(e / 9.0)
    ref = np.array([np.sum(a * np.cos(m * th)) for m in range(300)])
    assert np.abs(mu[0] - ref).max() <= TOL64


def test_moments_repeatable_and_profiled(T, ctx):
    lat = graphene(40, disorder_w=1.0, seed=1)
    T.tbpm_ctx_set_profiling(ctx.handle, True)
    try:
        a, _ = _gpu(T, ctx, lat, rho=9.0, num=257, seed=9)
        ms0, n0 = T.tbpm_ctx_kernel_time(ctx.handle, 0)
        ms1, n1 = T.tbpm_ctx_kernel_time(ctx.handle, 1)
    finally:
        T.tbpm_ctx_set_profiling(ctx.handle, False)
    b, _ = _gpu(T, ctx, lat, rho=9.0, num=257, seed=9)
    assert np.array_equal(a, b)                           # fixed reduction order
    assert n0 == 1 and n1 == 128                          # ceil(257 / 2) products with H
    assert ms0 > 0 and ms1 > 0


def test_moments_errors(T, ctx):
    lat = graphene(8)
    ham = ctx.build(lat)
    try:
        p, keep = T.make_params(9.0, 0, 1, sites=[0, 1])
        with pytest.raises(T.TBPMError) as ei:
            T.tbpm_chebyshev_moments(ctx.handle, ham, p, 10)
        assert ei.value.status == T.TBPM_ERR_ARG
        p, _ = T.make_params(5.0, 0, 1)
        with pytest.raises(T.TBPMError) as ei:
            T.tbpm_chebyshev_moments(ctx.handle, ham, p, 10)
        assert ei.value.status == T.TBPM_ERR_RESCALE
        p, _ = T.make_params(9.0, 0, 1)
        with pytest.raises(T.TBPMError) as ei:
            T.tbpm_chebyshev_moments(ctx.handle, ham, p, 0)
        assert ei.value.status == T.TBPM_ERR_ARG
        assert T.tbpm_moments_footprint(ham, p, 100) > 2 * lat.n * 16
    finally:
        T.tbpm_ham_destroy(ham)
