"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-only functions (Chebyshev coefficients, DOS transform, status
strings, argument checks) agree with the oracle.  No GPU call is made."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "tbpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(tbpm_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2509_26309_amd import tbpm
    return tbpm


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ["tbpm_build_csr", "tbpm_propagate_dos", "tbpm_submit", "tbpm_poll", "tbpm_dos",
                 "tbpm_ctx_create", "tbpm_server_create", "tbpm_coefficients"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    so = lib.load()
    missing = [n for n in _declared_functions() if not hasattr(so, n)]
    assert not missing, missing


def test_binding_wraps_every_symbol(lib):
    for n in _declared_functions():
        assert hasattr(lib, n), n


def test_coefficients_match_oracle(lib, orc):
    for tau, eps in [(np.pi, 1e-14), (0.5, 1e-14), (5.0, 1e-12), (30.0, 1e-13), (120.0, 1e-14)]:
        c = lib.tbpm_coefficients(tau, eps)
        o = orc.coefficients(tau, eps)
        assert c.size == o.size
        assert np.abs(c - o).max() < 1e-15


def test_coefficient_errors(lib):
    with pytest.raises(lib.TBPMError):
        lib.tbpm_coefficients(np.pi, 1e-14, max_terms=5)
    with pytest.raises(lib.TBPMError):
        lib.tbpm_coefficients(-1.0, 1e-14)


@pytest.mark.parametrize("window", [0, 1])
def test_dos_matches_oracle(lib, orc, window):
    rng = np.random.default_rng(3)
    for nt in [1, 7, 256]:
        c = rng.normal(size=nt + 1) + 1j * rng.normal(size=nt + 1)
        e, d = lib.tbpm_dos(c, 9.0, window)
        e2, d2 = orc.dos(c, 9.0, window)
        np.testing.assert_allclose(e, e2, rtol=0, atol=1e-14)
        np.testing.assert_allclose(d, d2, rtol=0, atol=1e-12)


def test_dos_argument_errors(lib):
    with pytest.raises(lib.TBPMError):
        lib.tbpm_dos(np.ones(1, dtype=complex), 9.0)
    with pytest.raises(lib.TBPMError):
        lib.tbpm_dos(np.ones(5, dtype=complex), -1.0)


def test_status_strings(lib):
    for s in range(-9, 2):
        assert lib.tbpm_status_string(s)
    assert lib.tbpm_status_string(lib.TBPM_ERR_RESCALE).startswith("rescale")


def test_no_gpu_fails_loudly(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except ImportError:
        pass
    with pytest.raises(lib.TBPMError):
        lib.tbpm_ctx_create(0)
