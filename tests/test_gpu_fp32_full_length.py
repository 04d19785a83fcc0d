"""Complex64 path over the full step counts of its workloads.

The complex64 path stores every Chebyshev iterate and the running series in
single precision (the paper names single precision only as future work, in
its summary); its bound against the FP64 oracle is max_k |dC| <= 1e-5 on
every C(t_k).  Rounding accumulates with the number of steps, so these
tests run reduced lattices from the same generators for the workloads'
own lengths:
  - AB bilayer + disorder W = 1 eV at 128 x 128 cells (65,536 orbitals, so the
    library picks the patch-reordered ELL it uses at full size), a block of 16
    vectors, 2048 steps; vectors 0 and 15 against the oracle, and the DOS of
    their mean;
  - 3rd-neighbour honeycomb with 1% vacancies at 96 x 96 cells, ELL, a block
    of 8 vectors, 4096 steps, the LDOS estimator at 64 sampled sites.
Every per-vector C(t) compared is held to 1e-5.

The LDOS estimator (n/R) sum_r conj(psi0_r[i]) psi_r(t)[i] is not averaged
over orbitals, so it sees in full the error of storing H in complex64: the
stored matrix is H + dH with |dH_ij| <= 2^-24 |H_ij|, so ||dH|| <= 2^-24 g
(g the Gershgorin bound), and by Duhamel's formula
||exp(-i(H+dH)t) - exp(-iHt)|| <= ||dH|| t.  Each estimator value sums R
terms of size n |psi0||psi| ~ 1, so against the FP64 oracle on H its bound
at t_k is 2^-24 g t_k + 10 x 1e-5 (the second part for the arithmetic, as in
the short parity tests).  Against the FP64 oracle on H rounded to complex64
(the matrix the path actually applies) only the arithmetic part remains:
10 x 1e-5.
"""
import copy

import numpy as np
import pytest

from tb_inputs import bilayer, honeycomb3, sample_sites

pytestmark = pytest.mark.gpu

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


def test_bilayer_block16_2048_steps(T, ctx, orc):
    lat = bilayer(128, disorder_w=1.0, seed=3)
    nt, R, rho = 2048, 16, 9.0
    ham = ctx.build(lat, dtype=T.TBPM_C64, fmt=T.TBPM_FMT_AUTO)
    try:
        assert T.tbpm_ham_info(ham)["format"] == T.TBPM_FMT_PATCH
        assert T.tbpm_ham_fused_pairs(ham, 16)
        p, _ = T.make_params(rho, nt, R, block=16, seed=3)
        out = T.tbpm_propagate_dos(ctx.handle, ham, p)
    finally:
        T.tbpm_ham_destroy(ham)
    rows = []
    for r in (0, 15):
        ref = orc.propagate(lat, orc.random_state(lat.n, 3, r), rescale=rho, num_steps=nt)
        err = float(np.abs(out["corr"][r] - ref.corr).max())
        nerr = float(np.abs(out["norms"][r] - ref.norms).max())
        print(f"bilayer 128^2 c64 B=16 {nt} steps: vector {r} max|dC| {err:.3e}, max|d norm| {nerr:.3e}")
        assert err <= TOL32, (r, err)
        assert nerr <= TOL32, (r, nerr)
        rows.append(ref.corr)
    # DOS of the two vectors' mean, GPU vs oracle
    _, d = T.tbpm_dos(out["corr"][[0, 15]].mean(axis=0), rho)
    _, d_ref = orc.dos(np.mean(rows, axis=0), rho)
    derr = float(np.abs(d - d_ref).max())
    print(f"bilayer 128^2 c64: max|dDOS| {derr:.3e}")
    assert derr <= TOL32


def test_honeycomb_vacancies_block8_4096_steps_ldos(T, ctx, orc):
    lat = honeycomb3(96, vacancy_p=0.01, seed=5)
    sites = sample_sites(lat.n, 64, 55)
    nt, R, rho = 4096, 8, 10.0
    ham = ctx.build(lat, dtype=T.TBPM_C64, fmt=T.TBPM_FMT_AUTO)
    try:
        assert T.tbpm_ham_info(ham)["format"] == T.TBPM_FMT_ELL
        p, keep = T.make_params(rho, nt, R, block=8, seed=5, sites=sites)
        out = T.tbpm_propagate_dos(ctx.handle, ham, p)
    finally:
        T.tbpm_ham_destroy(ham)
    # the same block on the patch format (the staged kernel)
    ham = ctx.build(lat, dtype=T.TBPM_C64, fmt=T.TBPM_FMT_PATCH)
    try:
        out_p = T.tbpm_propagate_dos(ctx.handle, ham, p)
    finally:
        T.tbpm_ham_destroy(ham)
    mean, per, norms, ld = orc.corr_dos(lat, rescale=rho, num_steps=nt, num_vectors=R, seed=5, sites=sites)
    perr = float(np.abs(out_p["corr"] - per).max())
    pnerr = float(np.abs(out_p["norms"] - norms).max())
    plerr = float(np.abs(out_p["ldos"] - ld).max())
    print(f"honeycomb 96^2 3NN vac c64 B=8 {nt} steps, patch format: max|dC| {perr:.3e}, "
          f"max|d norm| {pnerr:.3e}, LDOS max|d| {plerr:.3e}")
    assert perr <= TOL32
    assert pnerr <= TOL32
    err = float(np.abs(out["corr"] - per).max())
    nerr = float(np.abs(out["norms"] - norms).max())
    lerr = float(np.abs(out["ldos"] - ld).max())
    merr = float(np.abs(out["corr_mean"] - mean).max())
    assert merr <= TOL32
    _, d = T.tbpm_dos(out["corr_mean"], rho)
    _, d_ref = orc.dos(mean, rho)
    derr = float(np.abs(d - d_ref).max())
    print(f"honeycomb 96^2 3NN vac c64 B=8 {nt} steps: max|dC| {err:.3e}, max|d norm| {nerr:.3e}, "
          f"LDOS max|d| {lerr:.3e}, max|dDOS| {derr:.3e}")
    assert err <= TOL32
    assert nerr <= TOL32
    assert derr <= TOL32
    # LDOS estimator: the complex64 representation of H, bounded per time step
    g = orc.gershgorin(lat)
    t = np.arange(nt + 1) * np.pi / rho
    bound = 2.0 ** -24 * g * t + 10 * TOL32
    assert np.all(np.abs(out["ldos"] - ld) <= bound[None, :])
    assert np.all(np.abs(out_p["ldos"] - ld) <= bound[None, :])
    # ... and the arithmetic alone, against the oracle on the stored (rounded) matrix
    lat32 = copy.copy(lat)
    lat32.val = np.asarray(lat.val).astype(np.complex64).astype(np.complex128)
    _, per32, _, ld32 = orc.corr_dos(lat32, rescale=rho, num_steps=nt, num_vectors=R, seed=5, sites=sites)
    aerr = float(np.abs(out["ldos"] - ld32).max())
    cerr = float(np.abs(out["corr"] - per32).max())
    print(f"honeycomb 96^2 against the oracle on H rounded to complex64: max|dC| {cerr:.3e}, LDOS max|d| {aerr:.3e}")
    assert aerr <= 10 * TOL32
    assert cerr <= TOL32
