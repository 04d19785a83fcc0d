"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times, on sampled outputs the oracle can afford: the first time
steps of selected vectors.  Tolerances as in test_gpu_parity.py."""
import numpy as np
import pytest

from tb_inputs import graphene, bilayer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2509_26309_amd import tbpm
    return tbpm


@pytest.fixture(scope="module")
def ctx(T):
    c = T.Context(0)
    yield c
    c.close()


def test_graphene4096_disorder_fp64(T, ctx, orc):
    """33.5M orbitals, complex128, patch-reordered ELL with fused term pairs
    (chosen automatically, as in the benchmark), one vector at a time:
    vectors 0 and 3 for 2 steps against the oracle; norms for 24 steps."""
    lat = graphene(4096, disorder_w=1.0, seed=2)
    ham = ctx.build(lat, dtype=T.TBPM_C128, fmt=T.TBPM_FMT_AUTO)
    try:
        assert T.tbpm_ham_info(ham)["format"] == T.TBPM_FMT_PATCH
        for r in (0, 3):
            p, _ = T.make_params(9.0, 2, 1, block=1, seed=2, first_vector=r)
            out = T.tbpm_propagate_dos(ctx.handle, ham, p)
            ref = orc.propagate(lat, orc.random_state(lat.n, 2, r), rescale=9.0, num_steps=2)
            assert np.abs(out["corr"][0] - ref.corr).max() <= 1e-10
            assert np.abs(out["norms"][0] - ref.norms).max() <= 1e-10
        p, _ = T.make_params(9.0, 24, 1, block=1, seed=2)
        out = T.tbpm_propagate_dos(ctx.handle, ham, p)
        assert np.abs(out["norms"] - 1).max() <= 1e-12
        assert np.all(np.abs(out["corr"]) <= 1 + 1e-12)
    finally:
        T.tbpm_ham_destroy(ham)
    # the plain ELL path on the same workload
    ham = ctx.build(lat, dtype=T.TBPM_C128, fmt=T.TBPM_FMT_ELL)
    try:
        p, _ = T.make_params(9.0, 2, 1, block=1, seed=2, first_vector=0)
        out = T.tbpm_propagate_dos(ctx.handle, ham, p)
        ref = orc.propagate(lat, orc.random_state(lat.n, 2, 0), rescale=9.0, num_steps=2)
        assert np.abs(out["corr"][0] - ref.corr).max() <= 1e-10
    finally:
        T.tbpm_ham_destroy(ham)


def test_bilayer2048_fp32_block16(T, ctx, orc):
    """16.8M orbitals, complex64 SpMM of 16 vectors: vectors 0 and 15 for 2
    steps against the FP64 oracle; FP64 sums keep C(0) = 1 to 1e-6."""
    lat = bilayer(2048, disorder_w=1.0, seed=3)
    ham = ctx.build(lat, dtype=T.TBPM_C64, fmt=T.TBPM_FMT_AUTO)
    try:
        p, _ = T.make_params(9.0, 2, 16, block=16, seed=3)
        out = T.tbpm_propagate_dos(ctx.handle, ham, p)
        for r in (0, 15):
            ref = orc.propagate(lat, orc.random_state(lat.n, 3, r), rescale=9.0, num_steps=2)
            assert np.abs(out["corr"][r] - ref.corr).max() <= 1e-5
        assert np.abs(out["corr"][:, 0] - 1).max() <= 1e-6
    finally:
        T.tbpm_ham_destroy(ham)
