"""CPU oracle for the TBPM density-of-states path (FP64, plain loops).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark.  The GPU library and its Python binding
never import this package, and this package never imports them.

The arithmetic lives in tbpm_oracle.c (built into liboracle.so with gcc);
this module only marshals numpy arrays.  Every function follows TBPLaS 2.0,
section "Migration to C++" (Chebyshev series of the time-evolution operator
with the imaginary factor folded into the coefficients, three-term recurrence
formed in place as y <- 2 M x - y, then accumulated with its coefficient) and
section "Usage of TBPM solver" (random samples, rescale, number of time
steps, correlation function -> DOS).

Parity status of each function (pins in tests/test_oracle_*.py):
  splitmix64_next, phase_u, random_state  pinned (published SplitMix64 output
                                          sequence; phase statistics)
  coefficients                            pinned (Jacobi-Anger identity, sum rules)
  propagate (correlation, norms, sites)   pinned (exact diagonalization, Bloch sums,
                                          square-lattice closed form, unitarity)
  dos                                     pinned (discrete sum rule, single-level closed
                                          form, brute-force integral)
  gershgorin, is_hermitian                pinned (dense matrix checks)
  moments                                 pinned (exact diagonalization: sum |a_n|^2 T_m(E_n/rho))
  corr_from_moments                       pinned (exact diagonalization; agreement with propagate)
  kpm_dos                                 pinned (sum rule; Jackson kernel of a single level)
  propagate_outputs (snapshots, quasi-eigenstates)
                                          pinned (exact diagonalization; psi(0) and the final
                                          state of propagate; discrete orthogonality sum)
  fermi_coefficients                      pinned (the series against f(rho x) itself)
  response_corr                           pinned (exact diagonalization with exact f(E); limits
                                          mu far above / below the spectrum)
  ac_conductivity, dyn_polarization       pinned (a two-level correlation with a closed-form
                                          windowed sum; graphene's universal optical conductivity)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tbpm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over rows; no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_SRC) > os.path.getmtime(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, f64, u64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64
    lib.oracle_splitmix64_next.argtypes = [ctypes.POINTER(u64)]
    lib.oracle_splitmix64_next.restype = u64
    lib.oracle_phase_u.argtypes = [u64, i64, i64]
    lib.oracle_phase_u.restype = f64
    lib.oracle_random_state.argtypes = [i64, u64, i64, P]
    lib.oracle_random_state.restype = None
    lib.oracle_coefficients.argtypes = [f64, f64, ctypes.c_int, P]
    lib.oracle_coefficients.restype = ctypes.c_int
    lib.oracle_gershgorin.argtypes = [i64, P, P]
    lib.oracle_gershgorin.restype = f64
    lib.oracle_is_hermitian.argtypes = [i64, P, P, P, f64]
    lib.oracle_is_hermitian.restype = ctypes.c_int
    lib.oracle_propagate.argtypes = [i64, P, P, P, f64, f64, f64, ctypes.c_int, P, P, P, i64, P, P, P]
    lib.oracle_propagate.restype = ctypes.c_int
    lib.oracle_dos.argtypes = [P, ctypes.c_int, f64, ctypes.c_int, P, P]
    lib.oracle_dos.restype = ctypes.c_int
    lib.oracle_moments.argtypes = [i64, P, P, P, f64, P, ctypes.c_int, P]
    lib.oracle_moments.restype = ctypes.c_int
    lib.oracle_corr_from_moments.argtypes = [P, ctypes.c_int, ctypes.c_int, P]
    lib.oracle_corr_from_moments.restype = ctypes.c_int
    lib.oracle_kpm_dos.argtypes = [P, ctypes.c_int, f64, ctypes.c_int, P, P]
    lib.oracle_kpm_dos.restype = ctypes.c_int
    lib.oracle_propagate_outputs.argtypes = [i64, P, P, P, f64, f64, ctypes.c_int, P, ctypes.c_int, P, P,
                                             ctypes.c_int, P, P]
    lib.oracle_propagate_outputs.restype = ctypes.c_int
    lib.oracle_fermi_coefficients.argtypes = [f64, f64, f64, f64, ctypes.c_int, P]
    lib.oracle_fermi_coefficients.restype = ctypes.c_int
    lib.oracle_response_corr.argtypes = [i64, P, P, P, f64, f64, ctypes.c_int, P, P, P, P, P, P, P, f64, f64, f64, P]
    lib.oracle_response_corr.restype = ctypes.c_int
    lib.oracle_ac_conductivity.argtypes = [P, ctypes.c_int, f64, f64, f64, ctypes.c_int, P, P]
    lib.oracle_ac_conductivity.restype = ctypes.c_int
    lib.oracle_dyn_polarization.argtypes = [P, ctypes.c_int, f64, f64, ctypes.c_int, P, P]
    lib.oracle_dyn_polarization.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(threads: int) -> None:
    """Threads of the oracle's parallel loops (timing only; results do not change)."""
    _load().oracle_set_num_threads(int(threads))


def splitmix64_sequence(seed: int, count: int) -> np.ndarray:
    """The first `count` outputs of SplitMix64 seeded with `seed`."""
    lib = _load()
    st = ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF)
    return np.array([lib.oracle_splitmix64_next(ctypes.byref(st)) for _ in range(count)], dtype=np.uint64)


def phase_u(seed: int, r: int, i: int) -> float:
    """The uniform draw behind element i of random vector r (stream definition)."""
    return float(_load().oracle_phase_u(seed & 0xFFFFFFFFFFFFFFFF, r, i))


def random_state(n: int, seed: int, r: int = 0) -> np.ndarray:
    """psi0[i] = exp(2 pi i u_i) / sqrt(n) for random vector r."""
    out = np.empty(n, dtype=np.complex128)
    _load().oracle_random_state(n, seed & 0xFFFFFFFFFFFFFFFF, r, _ptr(out))
    return out


def coefficients(tau: float = np.pi, eps: float = 1e-14, max_terms: int = 4096) -> np.ndarray:
    """c_m = (2 - delta_m0) (-i)^m J_m(tau), m < M, truncated at |J_m| < eps past m > tau."""
    buf = np.zeros(max_terms, dtype=np.complex128)
    m = _load().oracle_coefficients(float(tau), float(eps), max_terms, _ptr(buf))
    if m < 0:
        raise ValueError("coefficient table too small")
    return buf[:m].copy()


def _csr(lat):
    rp = np.ascontiguousarray(lat.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(lat.col, dtype=np.int32)
    val = np.ascontiguousarray(lat.val, dtype=np.complex128)
    return rp, col, val


def gershgorin(lat) -> float:
    rp, col, val = _csr(lat)
    return float(_load().oracle_gershgorin(lat.n, _ptr(rp), _ptr(val)))


def is_hermitian(lat, tol: float = 1e-14) -> bool:
    rp, col, val = _csr(lat)
    return bool(_load().oracle_is_hermitian(lat.n, _ptr(rp), _ptr(col), _ptr(val), tol))


class PropagationResult:
    def __init__(self, corr, norms, site_corr, psi_final, num_terms):
        self.corr = corr              # complex128 [N_t + 1]
        self.norms = norms            # float64 [N_t + 1]
        self.site_corr = site_corr    # complex128 [sites, N_t + 1] or None
        self.psi_final = psi_final    # complex128 [n] or None
        self.num_terms = num_terms    # M


def propagate(lat, psi0: np.ndarray, *, rescale: float, num_steps: int, dt: Optional[float] = None,
              eps: float = 1e-14, sites: Optional[Sequence[int]] = None,
              keep_final: bool = False) -> PropagationResult:
    """Chebyshev propagation of psi0; C(t_k) = <psi0|psi(t_k)>, t_k = k dt, dt = pi/rescale."""
    rp, col, val = _csr(lat)
    psi0 = np.ascontiguousarray(psi0, dtype=np.complex128)
    if psi0.shape != (lat.n,):
        raise ValueError("psi0 has the wrong length")
    dt = np.pi / rescale if dt is None else float(dt)
    corr = np.zeros(num_steps + 1, dtype=np.complex128)
    norms = np.zeros(num_steps + 1, dtype=np.float64)
    s = None if sites is None else np.ascontiguousarray(sites, dtype=np.int64)
    ns = 0 if s is None else s.size
    site_corr = np.zeros((ns, num_steps + 1), dtype=np.complex128) if ns else None
    psi_final = np.zeros(lat.n, dtype=np.complex128) if keep_final else None
    m = _load().oracle_propagate(lat.n, _ptr(rp), _ptr(col), _ptr(val), float(rescale), dt, float(eps),
                                 int(num_steps), _ptr(psi0), _ptr(corr), _ptr(norms), ns, _ptr(s),
                                 _ptr(site_corr), _ptr(psi_final))
    if m == -2:
        raise ValueError("rescale is below the Gershgorin bound of H")
    if m < 0:
        raise RuntimeError(f"oracle_propagate failed ({m})")
    return PropagationResult(corr, norms, site_corr, psi_final, m)


def corr_dos(lat, *, rescale: float, num_steps: int, num_vectors: int = 1, seed: int = 1,
             eps: float = 1e-14, sites: Optional[Sequence[int]] = None, first_vector: int = 0):
    """Random-sample average of C(t) (and per-vector rows).

    Returns (mean corr [N_t+1], per-vector corr [R][N_t+1], norms [R][N_t+1],
    LDOS correlation [sites][N_t+1] or None) where the LDOS correlation is the
    estimator (N/R) sum_r conj(psi0_r[i]) psi_r(t)[i] at each site i.
    """
    rows, norms, ld = [], [], None
    for r in range(first_vector, first_vector + num_vectors):
        psi0 = random_state(lat.n, seed, r)
        res = propagate(lat, psi0, rescale=rescale, num_steps=num_steps, eps=eps, sites=sites)
        rows.append(res.corr)
        norms.append(res.norms)
        if res.site_corr is not None:
            ld = res.site_corr.copy() if ld is None else ld + res.site_corr
    per = np.array(rows)
    if ld is not None:
        ld = ld * (lat.n / num_vectors)
    return per.mean(axis=0), per, np.array(norms), ld


def dos(corr: np.ndarray, rescale: float, window: int = 1):
    """(energies [2 N_t], dos [2 N_t]) from C(t_k), k = 0..N_t."""
    corr = np.ascontiguousarray(corr, dtype=np.complex128)
    nt = corr.size - 1
    e = np.zeros(2 * nt)
    d = np.zeros(2 * nt)
    if _load().oracle_dos(_ptr(corr), nt, float(rescale), int(window), _ptr(e), _ptr(d)) != 0:
        raise ValueError("bad DOS arguments")
    return e, d


def moments(lat, psi0: np.ndarray, *, rescale: float, num_moments: int) -> np.ndarray:
    """mu_m = <psi0|T_m(H/rho)|psi0>, m < num_moments (plain recurrence), complex128."""
    rp, col, val = _csr(lat)
    psi0 = np.ascontiguousarray(psi0, dtype=np.complex128)
    mu = np.zeros(num_moments, dtype=np.complex128)
    r = _load().oracle_moments(lat.n, _ptr(rp), _ptr(col), _ptr(val), float(rescale), _ptr(psi0), int(num_moments),
                               _ptr(mu))
    if r == -2:
        raise ValueError("rescale is below the Gershgorin bound of H")
    if r != 0:
        raise RuntimeError(f"oracle_moments failed ({r})")
    return mu


def corr_from_moments(mu: np.ndarray, num_steps: int) -> np.ndarray:
    """C(t_k), k = 0..num_steps, t_k = k pi / rho, from Chebyshev moments."""
    mu = np.ascontiguousarray(mu, dtype=np.complex128)
    out = np.zeros(num_steps + 1, dtype=np.complex128)
    if _load().oracle_corr_from_moments(_ptr(mu), mu.size, int(num_steps), _ptr(out)) != 0:
        raise ValueError("bad arguments")
    return out


def kpm_dos(mu: np.ndarray, rescale: float, num_energies: int):
    """(energies, dos) of the Jackson-damped Chebyshev series at Chebyshev nodes."""
    mu = np.ascontiguousarray(mu, dtype=np.complex128)
    e = np.zeros(num_energies)
    d = np.zeros(num_energies)
    if _load().oracle_kpm_dos(_ptr(mu), mu.size, float(rescale), int(num_energies), _ptr(e), _ptr(d)) != 0:
        raise ValueError("bad arguments")
    return e, d


def propagate_outputs(lat, psi0: np.ndarray, *, rescale: float, num_steps: int, snap_steps=(), energies=(),
                      eps: float = 1e-14):
    """(snapshots [S, n], quasi-eigenstates [E, n]) of the propagation of psi0:
    psi(t_k) at the listed steps, and q_j = sum_k w_k exp(i E_j t_k) psi(t_k) (Hann w_k)."""
    rp, col, val = _csr(lat)
    psi0 = np.ascontiguousarray(psi0, dtype=np.complex128)
    st = np.ascontiguousarray(snap_steps, dtype=np.int32)
    en = np.ascontiguousarray(energies, dtype=np.float64)
    snaps = np.zeros((st.size, lat.n), dtype=np.complex128)
    qe = np.zeros((en.size, lat.n), dtype=np.complex128)
    r = _load().oracle_propagate_outputs(lat.n, _ptr(rp), _ptr(col), _ptr(val), float(rescale), float(eps),
                                         int(num_steps), _ptr(psi0), st.size, _ptr(st) if st.size else None,
                                         _ptr(snaps) if st.size else None, en.size,
                                         _ptr(en) if en.size else None, _ptr(qe) if en.size else None)
    if r == -2:
        raise ValueError("rescale is below the Gershgorin bound of H")
    if r < 0:
        raise RuntimeError(f"oracle_propagate_outputs failed ({r})")
    return snaps, qe


def fermi_coefficients(rescale: float, mu: float, kT: float, eps: float = 1e-14, max_terms: int = 16384):
    """Chebyshev coefficients a_m of the Fermi function f(rescale x), truncated at eps."""
    for cap in (256, 512, 1024, 2048, 4096, 8192, 16384):
        if cap > max_terms:
            break
        buf = np.zeros(cap)
        m = _load().oracle_fermi_coefficients(float(rescale), float(mu), float(kT), float(eps), cap, _ptr(buf))
        if m > 0:
            return buf[:m].copy()
    raise ValueError("Fermi series did not converge within max_terms")


def _op_csr(op):
    return (np.ascontiguousarray(op.row_ptr, dtype=np.int64), np.ascontiguousarray(op.col, dtype=np.int32),
            np.ascontiguousarray(op.val, dtype=np.complex128))


def response_corr(lat, phi: np.ndarray, a_op, b_op, *, rescale: float, num_steps: int, mu: float, kT: float,
                  eps: float = 1e-14, fermi_eps: float = 1e-14) -> np.ndarray:
    """corr(t_k) = <exp(-iHt) f(H) phi| A |exp(-iHt) (1 - f(H)) B phi>, k = 0..num_steps."""
    rp, col, val = _csr(lat)
    arp, acol, aval = _op_csr(a_op)
    brp, bcol, bval = _op_csr(b_op)
    phi = np.ascontiguousarray(phi, dtype=np.complex128)
    out = np.zeros(num_steps + 1, dtype=np.complex128)
    r = _load().oracle_response_corr(lat.n, _ptr(rp), _ptr(col), _ptr(val), float(rescale), float(eps),
                                     int(num_steps), _ptr(phi), _ptr(arp), _ptr(acol), _ptr(aval), _ptr(brp),
                                     _ptr(bcol), _ptr(bval), float(mu), float(kT), float(fermi_eps), _ptr(out))
    if r == -2:
        raise ValueError("rescale is below the Gershgorin bound of H")
    if r < 0:
        raise RuntimeError(f"oracle_response_corr failed ({r})")
    return out


def ac_conductivity(corr: np.ndarray, rescale: float, kT: float, omega_area: float, omegas) -> np.ndarray:
    corr = np.ascontiguousarray(corr, dtype=np.complex128)
    w = np.ascontiguousarray(omegas, dtype=np.float64)
    out = np.zeros(w.size)
    if _load().oracle_ac_conductivity(_ptr(corr), corr.size - 1, float(rescale), float(kT), float(omega_area),
                                      w.size, _ptr(w), _ptr(out)) != 0:
        raise ValueError("bad arguments")
    return out


def dyn_polarization(corr: np.ndarray, rescale: float, omega_area: float, omegas) -> np.ndarray:
    corr = np.ascontiguousarray(corr, dtype=np.complex128)
    w = np.ascontiguousarray(omegas, dtype=np.float64)
    out = np.zeros(w.size, dtype=np.complex128)
    if _load().oracle_dyn_polarization(_ptr(corr), corr.size - 1, float(rescale), float(omega_area), w.size,
                                       _ptr(w), _ptr(out)) != 0:
        raise ValueError("bad arguments")
    return out
