"""ctypes binding of libtbpm.so: the C ABI of include/tbpm.h under the same names.

Argument marshalling only: every step of the propagation runs in the HIP
library.  If libtbpm.so is not built, loading raises; nothing falls back to
the CPU.  Device memory can be served by PyTorch's caching allocator
(`TorchAllocator`) and the library can launch on a PyTorch stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtbpm.so")

TBPM_OK, TBPM_PENDING = 0, 1
TBPM_ERR_ARG, TBPM_ERR_CSR, TBPM_ERR_RESCALE, TBPM_ERR_TOO_LARGE = -1, -2, -3, -4
TBPM_ERR_OOM, TBPM_ERR_DIVERGED, TBPM_ERR_HIP, TBPM_ERR_CANCELLED, TBPM_ERR_UNKNOWN = -5, -6, -7, -8, -9
TBPM_C128, TBPM_C64 = 0, 1
TBPM_FMT_CSR, TBPM_FMT_ELL, TBPM_FMT_AUTO, TBPM_FMT_PATCH = 0, 1, 2, 3
TBPM_BUILD_CHECK_HERMITIAN, TBPM_BUILD_LARGE_PATCHES, TBPM_BUILD_NO_VALUE_TABLE = 1, 2, 4
TBPM_SERIES_FORWARD, TBPM_SERIES_CLENSHAW = 0, 1

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class tbpm_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class tbpm_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class tbpm_params(ctypes.Structure):
    _fields_ = [("rescale", ctypes.c_double), ("num_time_steps", ctypes.c_int32),
                ("num_vectors", ctypes.c_int32), ("block", ctypes.c_int32), ("first_vector", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("bessel_eps", ctypes.c_double), ("norm_tol", ctypes.c_double),
                ("ldos_sites", ctypes.c_void_p), ("num_ldos_sites", ctypes.c_int32),
                ("lanes_per_row", ctypes.c_int32)]


class TBPMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


_lib = None
P = ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)
_SIGS = {
    "tbpm_status_string": ([ctypes.c_int32], ctypes.c_char_p),
    "tbpm_last_error": ([P], ctypes.c_char_p),
    "tbpm_ctx_create": ([ctypes.c_int, ctypes.POINTER(tbpm_allocator), P, PP], ctypes.c_int32),
    "tbpm_ctx_destroy": ([P], ctypes.c_int32),
    "tbpm_ctx_set_profiling": ([P, ctypes.c_int32], ctypes.c_int32),
    "tbpm_ctx_kernel_time": ([P, ctypes.c_int32, P, P], ctypes.c_int32),
    "tbpm_ctx_set_graphs": ([P, ctypes.c_int32], ctypes.c_int32),
    "tbpm_ctx_graph_replays": ([P, P], ctypes.c_int32),
    "tbpm_ctx_set_series": ([P, ctypes.c_int32], ctypes.c_int32),
    "tbpm_build_csr": ([P, ctypes.POINTER(tbpm_csr), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, PP],
                       ctypes.c_int32),
    "tbpm_ham_info": ([P, P, P, P, P, P, P], ctypes.c_int32),
    "tbpm_ham_destroy": ([P], ctypes.c_int32),
    "tbpm_footprint": ([P, ctypes.POINTER(tbpm_params), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int32),
    "tbpm_autotune": ([P, P, ctypes.c_int32, P, P, P], ctypes.c_int32),
    "tbpm_ham_set_tuning": ([P, ctypes.c_int32, ctypes.c_int32], ctypes.c_int32),
    "tbpm_patch_plan": ([ctypes.POINTER(tbpm_csr), ctypes.c_int32, P, P, P, P], ctypes.c_int32),
    "tbpm_ham_value_table": ([P, P, P], ctypes.c_int32),
    "tbpm_ham_fused_pairs": ([P, ctypes.c_int32, P], ctypes.c_int32),
    "tbpm_value_table_plan": ([ctypes.POINTER(tbpm_csr), ctypes.c_int32, P, P], ctypes.c_int32),
    "tbpm_coefficients": ([ctypes.c_double, ctypes.c_double, ctypes.c_int32, P, P], ctypes.c_int32),
    "tbpm_propagate_dos": ([P, P, ctypes.POINTER(tbpm_params), P, P, P, P], ctypes.c_int32),
    "tbpm_propagate_dos_noalloc": ([P, P, ctypes.POINTER(tbpm_params), P, P, P], ctypes.c_int32),
    "tbpm_propagate_states": ([P, P, ctypes.POINTER(tbpm_params), P, P, P, P], ctypes.c_int32),
    "tbpm_dos": ([P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, P, P], ctypes.c_int32),
    "tbpm_sample_mean": ([P, ctypes.c_int32, ctypes.c_int32, P], ctypes.c_int32),
    "tbpm_chebyshev_moments": ([P, P, ctypes.POINTER(tbpm_params), ctypes.c_int32, P], ctypes.c_int32),
    "tbpm_time_evolution": ([P, P, ctypes.POINTER(tbpm_params), P, ctypes.c_int32, P, P, P], ctypes.c_int32),
    "tbpm_propagate_sites": ([P, P, ctypes.POINTER(tbpm_params), P, ctypes.c_int32, P, P], ctypes.c_int32),
    "tbpm_site_moments": ([P, P, ctypes.POINTER(tbpm_params), P, ctypes.c_int32, ctypes.c_int32, P],
                          ctypes.c_int32),
    "tbpm_quasi_eigenstates": ([P, P, ctypes.POINTER(tbpm_params), P, ctypes.c_int32, P, P, P], ctypes.c_int32),
    "tbpm_moments_footprint": ([P, ctypes.POINTER(tbpm_params), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
                               ctypes.c_int32),
    "tbpm_moments_needed": ([ctypes.c_int32, ctypes.c_double, P], ctypes.c_int32),
    "tbpm_corr_from_moments": ([P, ctypes.c_int32, ctypes.c_int32, P], ctypes.c_int32),
    "tbpm_kpm_dos": ([P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, P, P], ctypes.c_int32),
    "tbpm_build_operator": ([P, P, ctypes.POINTER(tbpm_csr), PP], ctypes.c_int32),
    "tbpm_response_corr": ([P, P, P, P, ctypes.POINTER(tbpm_params), ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, P], ctypes.c_int32),
    "tbpm_fermi_coefficients": ([ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int32, P, P], ctypes.c_int32),
    "tbpm_ac_conductivity": ([P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_int32, P, P], ctypes.c_int32),
    "tbpm_dyn_polarization": ([P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32, P, P],
                              ctypes.c_int32),
    "tbpm_server_create": ([P, ctypes.c_size_t, ctypes.c_int32, PP], ctypes.c_int32),
    "tbpm_submit": ([P, P, ctypes.POINTER(tbpm_params), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int32),
    "tbpm_poll": ([P, ctypes.c_uint64, P, ctypes.c_int64, P, ctypes.c_int64, P], ctypes.c_int32),
    "tbpm_cancel": ([P, ctypes.c_uint64], ctypes.c_int32),
    "tbpm_server_destroy": ([P], ctypes.c_int32),
}


def load() -> ctypes.CDLL:
    """Loads libtbpm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2509_26309_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def tbpm_status_string(s: int) -> str:
    return load().tbpm_status_string(s).decode()


def tbpm_last_error(ctx) -> str:
    return load().tbpm_last_error(ctx).decode()


def _check(status: int, ctx=None, what: str = "") -> int:
    if status < 0:
        msg = tbpm_status_string(status)
        if ctx is not None:
            detail = tbpm_last_error(ctx)
            if detail:
                msg = f"{msg}: {detail}"
        raise TBPMError(status, f"{what}: {msg}" if what else msg)
    return status


# ---- allocators -------------------------------------------------------------------

class TorchAllocator:
    """Serves the library's device memory from PyTorch's caching allocator."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self._device = device
        self._live = {}

        self.calls = 0

        def _alloc(nbytes, user):
            self.calls += 1
            try:
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{device}")
            except Exception:
                return None
            p = t.data_ptr()
            self._live[p] = t
            return p

        def _free(ptr, user):
            if ptr:
                self._live.pop(int(ptr), None)

        self._alloc_cb = ALLOC_FN(_alloc)
        self._free_cb = FREE_FN(_free)
        self.struct = tbpm_allocator(self._alloc_cb, self._free_cb, None)

    @property
    def live_bytes(self) -> int:
        return sum(t.numel() for t in self._live.values())


# ---- C functions (same names) ---------------------------------------------------------

def tbpm_ctx_create(device: int = 0, allocator: Optional[TorchAllocator] = None, hip_stream: Optional[int] = None):
    out = ctypes.c_void_p()
    a = ctypes.byref(allocator.struct) if allocator is not None else None
    _check(load().tbpm_ctx_create(device, a, ctypes.c_void_p(hip_stream) if hip_stream else None,
                                  ctypes.byref(out)), what="tbpm_ctx_create")
    return out


def tbpm_ctx_destroy(ctx) -> None:
    _check(load().tbpm_ctx_destroy(ctx), what="tbpm_ctx_destroy")


def tbpm_ctx_set_profiling(ctx, enable: bool) -> None:
    _check(load().tbpm_ctx_set_profiling(ctx, 1 if enable else 0), what="tbpm_ctx_set_profiling")


def tbpm_ctx_set_graphs(ctx, mode: int) -> None:
    _check(load().tbpm_ctx_set_graphs(ctx, int(mode)), what="tbpm_ctx_set_graphs")


def tbpm_ctx_set_series(ctx, mode: int) -> None:
    _check(load().tbpm_ctx_set_series(ctx, int(mode)), what="tbpm_ctx_set_series")


def tbpm_ctx_graph_replays(ctx) -> int:
    n = ctypes.c_int64()
    _check(load().tbpm_ctx_graph_replays(ctx, ctypes.byref(n)), what="tbpm_ctx_graph_replays")
    return n.value


def tbpm_ctx_kernel_time(ctx, kind: int):
    """(total milliseconds, launches) timed for kind 0 first / 1 middle / 2 last term."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load().tbpm_ctx_kernel_time(ctx, kind, ctypes.byref(ms), ctypes.byref(n)), what="tbpm_ctx_kernel_time")
    return ms.value, n.value


def tbpm_build_csr(ctx, n: int, row_ptr: np.ndarray, col: np.ndarray, val: np.ndarray, dtype: int = TBPM_C128,
                   fmt: int = TBPM_FMT_AUTO, flags: int = 0):
    """row_ptr int64 [n+1], col int32 [nnz], val complex128 [nnz] in host memory."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    vl = np.ascontiguousarray(val, dtype=np.complex128)
    csr = tbpm_csr(int(n), int(rp[-1]) if rp.size else 0, rp.ctypes.data, cl.ctypes.data, vl.ctypes.data, 0)
    out = ctypes.c_void_p()
    _check(load().tbpm_build_csr(ctx, ctypes.byref(csr), dtype, fmt, flags, ctypes.byref(out)), ctx,
           "tbpm_build_csr")
    return out


def tbpm_build_csr_device(ctx, n: int, nnz: int, row_ptr_ptr: int, col_ptr: int, val_ptr: int,
                          dtype: int = TBPM_C128, fmt: int = TBPM_FMT_AUTO, flags: int = 0):
    """tbpm_build_csr on arrays already in device memory (int64 / int32 / complex128)."""
    csr = tbpm_csr(int(n), int(nnz), row_ptr_ptr, col_ptr, val_ptr, 1)
    out = ctypes.c_void_p()
    _check(load().tbpm_build_csr(ctx, ctypes.byref(csr), dtype, fmt, flags, ctypes.byref(out)), ctx,
           "tbpm_build_csr")
    return out


def tbpm_ham_info(ham) -> dict:
    n, nnz = ctypes.c_int64(), ctypes.c_int64()
    g = ctypes.c_double()
    b = ctypes.c_size_t()
    dt, fm = ctypes.c_int32(), ctypes.c_int32()
    _check(load().tbpm_ham_info(ham, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(g), ctypes.byref(b),
                                ctypes.byref(dt), ctypes.byref(fm)), what="tbpm_ham_info")
    return {"n": n.value, "nnz": nnz.value, "gershgorin": g.value, "bytes": b.value, "dtype": dt.value,
            "format": fm.value}


def tbpm_ham_value_table(ham) -> dict:
    """Entries of the stored value table (0: none) and how the diagonal is kept: 0 in the table,
    1 per row, 2 per row as real parts."""
    e, d = ctypes.c_int32(), ctypes.c_int32()
    _check(load().tbpm_ham_value_table(ham, ctypes.byref(e), ctypes.byref(d)), what="tbpm_ham_value_table")
    return {"entries": e.value, "per_row_diagonal": d.value}


def tbpm_ham_fused_pairs(ham, block: int) -> bool:
    """Whether the forward recurrence runs the middle terms of blocks of `block` vectors two to a launch."""
    f = ctypes.c_int32()
    _check(load().tbpm_ham_fused_pairs(ham, int(block), ctypes.byref(f)), what="tbpm_ham_fused_pairs")
    return bool(f.value)


def tbpm_value_table_plan(n: int, row_ptr: np.ndarray, col: np.ndarray, val: np.ndarray,
                          dtype: int = TBPM_C128) -> dict:
    """Host-only: the value table tbpm_build_csr would store for this CSR."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    vl = np.ascontiguousarray(val, dtype=np.complex128)
    csr = tbpm_csr(int(n), int(rp[-1]), rp.ctypes.data, cl.ctypes.data, vl.ctypes.data, 0)
    e, d = ctypes.c_int32(), ctypes.c_int32()
    _check(load().tbpm_value_table_plan(ctypes.byref(csr), int(dtype), ctypes.byref(e), ctypes.byref(d)),
           what="tbpm_value_table_plan")
    return {"entries": e.value, "per_row_diagonal": d.value}


def tbpm_ham_destroy(ham) -> None:
    _check(load().tbpm_ham_destroy(ham), what="tbpm_ham_destroy")


def make_params(rescale: float, num_time_steps: int, num_vectors: int = 1, *, block: int = 0, first_vector: int = 0,
                seed: int = 1, bessel_eps: float = 1e-14, norm_tol: float = 0.0,
                sites: Optional[Sequence[int]] = None, lanes_per_row: int = 0):
    """tbpm_params plus the keep-alive array of LDOS sites."""
    s = None if sites is None else np.ascontiguousarray(sites, dtype=np.int64)
    p = tbpm_params(float(rescale), int(num_time_steps), int(num_vectors), int(block), int(first_vector),
                    int(seed) & 0xFFFFFFFFFFFFFFFF, float(bessel_eps), float(norm_tol),
                    None if s is None else s.ctypes.data, 0 if s is None else int(s.size), int(lanes_per_row))
    return p, s


def tbpm_autotune(ctx, ham, max_block: int = 16) -> dict:
    """Times the candidate shapes of the middle term and stores the best in `ham`."""
    lanes, block = ctypes.c_int32(), ctypes.c_int32()
    us = ctypes.c_double()
    _check(load().tbpm_autotune(ctx, ham, int(max_block), ctypes.byref(lanes), ctypes.byref(block),
                                ctypes.byref(us)), ctx, "tbpm_autotune")
    return {"lanes_per_row": lanes.value, "block": block.value, "us_per_vector_term": us.value}


def tbpm_patch_plan(n: int, row_ptr: np.ndarray, col: np.ndarray, patch_rows: int = 1024) -> dict:
    """Host-only: the patch reordering the library would apply (new index of each row and halo statistics)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    csr = tbpm_csr(int(n), int(rp[-1]), rp.ctypes.data, cl.ctypes.data, None, 0)
    new = np.zeros(n, dtype=np.int32)
    npatch = ctypes.c_int64()
    mh = ctypes.c_int32()
    hf = ctypes.c_double()
    _check(load().tbpm_patch_plan(ctypes.byref(csr), int(patch_rows), _ptr(new), ctypes.byref(npatch),
                                  ctypes.byref(mh), ctypes.byref(hf)), what="tbpm_patch_plan")
    return {"new_of_old": new, "num_patches": npatch.value, "max_halo": mh.value, "halo_fraction": hf.value}


def tbpm_ham_set_tuning(ham, lanes_per_row: int, block: int) -> None:
    _check(load().tbpm_ham_set_tuning(ham, int(lanes_per_row), int(block)), what="tbpm_ham_set_tuning")


def autotune_cached(ctx, ham, key: str, max_block: int = 16, path: Optional[str] = None) -> dict:
    """tbpm_autotune with a persisted cache: results are stored in a JSON file
    under `key` (describe the matrix: shape, nnz, dtype, format) and reused."""
    import json
    path = path or os.environ.get("TBPM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                                 "tbpm_autotune.json"))
    full = f"{key}|max_block={max_block}"
    cache = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if full in cache:
        r = cache[full]
        tbpm_ham_set_tuning(ham, r["lanes_per_row"], r["block"])
        return dict(r, cached=True)
    r = tbpm_autotune(ctx, ham, max_block)
    cache[full] = r
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1)
    os.replace(tmp, path)
    return dict(r, cached=False)


def tbpm_footprint(ham, params: tbpm_params) -> int:
    b = ctypes.c_size_t()
    _check(load().tbpm_footprint(ham, ctypes.byref(params), ctypes.byref(b)), what="tbpm_footprint")
    return b.value


def tbpm_coefficients(tau: float, eps: float = 1e-14, max_terms: int = 4096) -> np.ndarray:
    buf = np.zeros(max_terms, dtype=np.complex128)
    m = ctypes.c_int32()
    _check(load().tbpm_coefficients(float(tau), float(eps), max_terms, _ptr(buf), ctypes.byref(m)),
           what="tbpm_coefficients")
    return buf[:m.value].copy()


def tbpm_propagate_dos(ctx, ham, params: tbpm_params, *, want_norms: bool = True, want_rows: bool = True) -> dict:
    """calc_corr_dos: {"corr_mean": sample average C(t_k) [N_t+1], "corr": per-vector
    C_r(t_k) [R][N_t+1] (None unless want_rows), "norms", "ldos", "status"}."""
    R, nt1 = params.num_vectors, params.num_time_steps + 1
    corr = np.zeros((R, nt1), dtype=np.complex128) if want_rows else None
    norms = np.zeros((R, nt1), dtype=np.float64) if want_norms else None
    ldos = np.zeros((params.num_ldos_sites, nt1), dtype=np.complex128) if params.num_ldos_sites > 0 else None
    mean = np.zeros(nt1, dtype=np.complex128)
    st = load().tbpm_propagate_dos(ctx, ham, ctypes.byref(params), _ptr(corr), _ptr(norms), _ptr(ldos), _ptr(mean))
    out = {"corr": corr, "norms": norms, "ldos": ldos, "corr_mean": mean, "status": st}
    if st == TBPM_ERR_DIVERGED:
        out["error"] = tbpm_last_error(ctx)
        return out
    _check(st, ctx, "tbpm_propagate_dos")
    return out


TBPM_NOALLOC_MAX_BYTES = 64 << 20


def tbpm_propagate_dos_noalloc(ctx, ham, params: tbpm_params, *, want_norms: bool = True) -> dict:
    """tbpm_propagate_dos with every device buffer in the library's fixed scratch
    area (no device allocation): {"corr", "norms", "corr_mean", "status"}."""
    R, nt1 = params.num_vectors, params.num_time_steps + 1
    corr = np.zeros((R, nt1), dtype=np.complex128)
    norms = np.zeros((R, nt1), dtype=np.float64) if want_norms else None
    mean = np.zeros(nt1, dtype=np.complex128)
    st = load().tbpm_propagate_dos_noalloc(ctx, ham, ctypes.byref(params), _ptr(corr), _ptr(norms), _ptr(mean))
    out = {"corr": corr, "norms": norms, "corr_mean": mean, "status": st}
    if st == TBPM_ERR_DIVERGED:
        out["error"] = tbpm_last_error(ctx)
        return out
    _check(st, ctx, "tbpm_propagate_dos_noalloc")
    return out


def tbpm_propagate_states(ctx, ham, params: tbpm_params, psi0: np.ndarray, *, keep_final: bool = False) -> dict:
    psi0 = np.ascontiguousarray(np.atleast_2d(psi0), dtype=np.complex128)
    R, nt1 = params.num_vectors, params.num_time_steps + 1
    if psi0.shape[0] != R:
        raise ValueError("psi0 must hold num_vectors rows")
    corr = np.zeros((R, nt1), dtype=np.complex128)
    norms = np.zeros((R, nt1), dtype=np.float64)
    fin = np.zeros_like(psi0) if keep_final else None
    st = load().tbpm_propagate_states(ctx, ham, ctypes.byref(params), _ptr(psi0), _ptr(corr), _ptr(norms), _ptr(fin))
    _check(st, ctx, "tbpm_propagate_states")
    return {"corr": corr, "norms": norms, "psi_final": fin}


def tbpm_sample_mean(rows: np.ndarray) -> np.ndarray:
    """(1/R) sum_r rows[r] of complex rows [R][len], summed by the library in order r = 0..R-1."""
    rows = np.ascontiguousarray(rows, dtype=np.complex128)
    if rows.ndim != 2:
        raise ValueError("rows must be two-dimensional")
    mean = np.zeros(rows.shape[1], dtype=np.complex128)
    _check(load().tbpm_sample_mean(_ptr(rows), rows.shape[0], rows.shape[1], _ptr(mean)), what="tbpm_sample_mean")
    return mean


def tbpm_dos(corr: np.ndarray, rescale: float, window: int = 1):
    corr = np.ascontiguousarray(corr, dtype=np.complex128)
    nt = corr.size - 1
    e = np.zeros(2 * nt)
    d = np.zeros(2 * nt)
    _check(load().tbpm_dos(_ptr(corr), nt, float(rescale), int(window), _ptr(e), _ptr(d)), what="tbpm_dos")
    return e, d


def tbpm_propagate_sites(ctx, ham, params: tbpm_params, sites) -> dict:
    """Exact local correlation C_i(t_k) = <i|e^{-iHt_k}|i> per site (complex128 [S, N_t+1]) and norms."""
    s = np.ascontiguousarray(sites, dtype=np.int64).ravel()
    nt1 = params.num_time_steps + 1
    corr = np.zeros((s.size, nt1), dtype=np.complex128)
    norms = np.zeros((s.size, nt1), dtype=np.float64)
    _check(load().tbpm_propagate_sites(ctx, ham, ctypes.byref(params), _ptr(s), s.size, _ptr(corr), _ptr(norms)),
           ctx, "tbpm_propagate_sites")
    return {"corr": corr, "norms": norms}


def tbpm_site_moments(ctx, ham, params: tbpm_params, sites, num_moments: int) -> np.ndarray:
    """mu[s, m] = <i_s|T_m(H/rescale)|i_s>, complex128 [S, num_moments]."""
    s = np.ascontiguousarray(sites, dtype=np.int64).ravel()
    mu = np.zeros((s.size, int(num_moments)), dtype=np.complex128)
    _check(load().tbpm_site_moments(ctx, ham, ctypes.byref(params), _ptr(s), s.size, int(num_moments), _ptr(mu)),
           ctx, "tbpm_site_moments")
    return mu


def _one_state(psi0, n):
    if psi0 is None:
        return None
    psi0 = np.ascontiguousarray(psi0, dtype=np.complex128).ravel()
    if psi0.size != n:
        raise ValueError("psi0 must hold n complex values")
    return psi0


def tbpm_time_evolution(ctx, ham, params: tbpm_params, steps, psi0: Optional[np.ndarray] = None) -> dict:
    """psi(t_k) at the listed steps (complex128 [S, n], original row order) and C(t)."""
    n = tbpm_ham_info(ham)["n"]
    psi0 = _one_state(psi0, n)
    st = np.ascontiguousarray(steps, dtype=np.int32).ravel()
    snaps = np.zeros((st.size, n), dtype=np.complex128)
    corr = np.zeros(params.num_time_steps + 1, dtype=np.complex128)
    _check(load().tbpm_time_evolution(ctx, ham, ctypes.byref(params), _ptr(psi0), st.size, _ptr(st), _ptr(snaps),
                                      _ptr(corr)), ctx, "tbpm_time_evolution")
    return {"snapshots": snaps, "corr": corr}


def tbpm_quasi_eigenstates(ctx, ham, params: tbpm_params, energies, psi0: Optional[np.ndarray] = None) -> dict:
    """Unnormalised quasi-eigenstates (complex128 [E, n], original row order) and C(t)."""
    n = tbpm_ham_info(ham)["n"]
    psi0 = _one_state(psi0, n)
    en = np.ascontiguousarray(energies, dtype=np.float64).ravel()
    qe = np.zeros((en.size, n), dtype=np.complex128)
    corr = np.zeros(params.num_time_steps + 1, dtype=np.complex128)
    _check(load().tbpm_quasi_eigenstates(ctx, ham, ctypes.byref(params), _ptr(psi0), en.size, _ptr(en), _ptr(qe),
                                         _ptr(corr)), ctx, "tbpm_quasi_eigenstates")
    return {"qe": qe, "corr": corr}


def tbpm_chebyshev_moments(ctx, ham, params: tbpm_params, num_moments: int) -> np.ndarray:
    """mu[r, m] = <psi0_r|T_m(H/rescale)|psi0_r>, complex128 [R, num_moments]."""
    mu = np.zeros((params.num_vectors, int(num_moments)), dtype=np.complex128)
    _check(load().tbpm_chebyshev_moments(ctx, ham, ctypes.byref(params), int(num_moments), _ptr(mu)), ctx,
           "tbpm_chebyshev_moments")
    return mu


def tbpm_moments_footprint(ham, params: tbpm_params, num_moments: int) -> int:
    b = ctypes.c_size_t()
    _check(load().tbpm_moments_footprint(ham, ctypes.byref(params), int(num_moments), ctypes.byref(b)),
           what="tbpm_moments_footprint")
    return b.value


def tbpm_moments_needed(num_time_steps: int, eps: float = 1e-14) -> int:
    m = ctypes.c_int32()
    _check(load().tbpm_moments_needed(int(num_time_steps), float(eps), ctypes.byref(m)), what="tbpm_moments_needed")
    return m.value


def tbpm_corr_from_moments(mu: np.ndarray, num_time_steps: int) -> np.ndarray:
    mu = np.ascontiguousarray(mu, dtype=np.complex128).ravel()
    corr = np.zeros(int(num_time_steps) + 1, dtype=np.complex128)
    _check(load().tbpm_corr_from_moments(_ptr(mu), mu.size, int(num_time_steps), _ptr(corr)),
           what="tbpm_corr_from_moments")
    return corr


def tbpm_kpm_dos(mu: np.ndarray, rescale: float, num_energies: int):
    mu = np.ascontiguousarray(mu, dtype=np.complex128).ravel()
    e = np.zeros(int(num_energies))
    d = np.zeros(int(num_energies))
    _check(load().tbpm_kpm_dos(_ptr(mu), mu.size, float(rescale), int(num_energies), _ptr(e), _ptr(d)),
           what="tbpm_kpm_dos")
    return e, d


def tbpm_build_operator(ctx, ham, n: int, row_ptr: np.ndarray, col: np.ndarray, val: np.ndarray):
    """Stores an operator (host CSR) in ham's dtype and row order; returns its handle."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.complex128)
    csr = tbpm_csr(int(n), int(rp[-1]), rp.ctypes.data, c.ctypes.data, v.ctypes.data, 0)
    out = ctypes.c_void_p()
    _check(load().tbpm_build_operator(ctx, ham, ctypes.byref(csr), ctypes.byref(out)), ctx, "tbpm_build_operator")
    return out


def tbpm_response_corr(ctx, ham, op_a, op_b, params: tbpm_params, mu: float, kT: float,
                       fermi_eps: float = 1e-14) -> np.ndarray:
    """corr[r, k] = <exp(-iHt_k) f(H) phi_r| A |exp(-iHt_k) (1 - f(H)) B phi_r>, complex128 [R, N_t+1]."""
    corr = np.zeros((params.num_vectors, params.num_time_steps + 1), dtype=np.complex128)
    _check(load().tbpm_response_corr(ctx, ham, op_a, op_b, ctypes.byref(params), float(mu), float(kT),
                                     float(fermi_eps), _ptr(corr)), ctx, "tbpm_response_corr")
    return corr


def tbpm_fermi_coefficients(rescale: float, mu: float, kT: float, eps: float = 1e-14,
                            max_terms: int = 1 << 20) -> np.ndarray:
    buf = np.zeros(max_terms)
    m = ctypes.c_int32()
    _check(load().tbpm_fermi_coefficients(float(rescale), float(mu), float(kT), float(eps), max_terms, _ptr(buf),
                                          ctypes.byref(m)), what="tbpm_fermi_coefficients")
    return buf[:m.value].copy()


def tbpm_ac_conductivity(corr: np.ndarray, rescale: float, kT: float, area_per_orbital: float, omegas) -> np.ndarray:
    corr = np.ascontiguousarray(corr, dtype=np.complex128).ravel()
    w = np.ascontiguousarray(omegas, dtype=np.float64).ravel()
    out = np.zeros(w.size)
    _check(load().tbpm_ac_conductivity(_ptr(corr), corr.size - 1, float(rescale), float(kT), float(area_per_orbital),
                                       w.size, _ptr(w), _ptr(out)), what="tbpm_ac_conductivity")
    return out


def tbpm_dyn_polarization(corr: np.ndarray, rescale: float, area_per_orbital: float, omegas) -> np.ndarray:
    corr = np.ascontiguousarray(corr, dtype=np.complex128).ravel()
    w = np.ascontiguousarray(omegas, dtype=np.float64).ravel()
    out = np.zeros(w.size, dtype=np.complex128)
    _check(load().tbpm_dyn_polarization(_ptr(corr), corr.size - 1, float(rescale), float(area_per_orbital), w.size,
                                        _ptr(w), _ptr(out)), what="tbpm_dyn_polarization")
    return out


def tbpm_server_create(ctx, hbm_budget: int, max_slots: int):
    out = ctypes.c_void_p()
    _check(load().tbpm_server_create(ctx, int(hbm_budget), int(max_slots), ctypes.byref(out)), ctx,
           "tbpm_server_create")
    return out


def tbpm_submit(srv, ham, params: tbpm_params) -> int:
    t = ctypes.c_uint64()
    _check(load().tbpm_submit(srv, ham, ctypes.byref(params), ctypes.byref(t)), what="tbpm_submit")
    return t.value


def tbpm_poll(srv, ticket: int, num_vectors: int, num_time_steps: int):
    """(status, corr [R][N_t+1] or None, timings (submit, admit, done), sample mean [N_t+1] or None).
    num_vectors and num_time_steps size the output buffers; the library
    rejects buffers smaller than the submitted request's (TBPM_ERR_ARG)."""
    corr = np.zeros((num_vectors, num_time_steps + 1), dtype=np.complex128)
    mean = np.zeros(num_time_steps + 1, dtype=np.complex128)
    tm = np.zeros(3)
    st = load().tbpm_poll(srv, ctypes.c_uint64(ticket), _ptr(corr), corr.size, _ptr(mean), mean.size, _ptr(tm))
    if st < 0 and st not in (TBPM_ERR_CANCELLED, TBPM_ERR_DIVERGED, TBPM_ERR_OOM, TBPM_ERR_HIP):
        _check(st, what="tbpm_poll")
    ok = st == TBPM_OK
    return st, (corr if ok else None), tm, (mean if ok else None)


def tbpm_cancel(srv, ticket: int) -> None:
    _check(load().tbpm_cancel(srv, ctypes.c_uint64(ticket)), what="tbpm_cancel")


def tbpm_server_destroy(srv) -> None:
    _check(load().tbpm_server_destroy(srv), what="tbpm_server_destroy")


# ---- convenience ------------------------------------------------------------------------

class Context:
    """A tbpm_ctx on `device`, with memory from PyTorch (default) or hipMalloc and,
    by default, launching on PyTorch's current stream."""

    def __init__(self, device: int = 0, allocator: str = "torch", torch_stream: bool = True):
        self.allocator = None
        stream = None
        if allocator not in ("torch", "hip"):
            raise ValueError("allocator must be 'torch' or 'hip'")
        if allocator == "torch" or torch_stream:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU visible to PyTorch")
            torch.cuda.set_device(device)
            if allocator == "torch":
                self.allocator = TorchAllocator(device)
            if torch_stream:
                stream = torch.cuda.current_stream(device).cuda_stream
        self.handle = tbpm_ctx_create(device, self.allocator, stream)

    def build(self, lat, dtype: int = TBPM_C128, fmt: int = TBPM_FMT_AUTO, check_hermitian: bool = False,
              flags: int = 0):
        return tbpm_build_csr(self.handle, lat.n, lat.row_ptr, lat.col, lat.val, dtype, fmt,
                              flags | (TBPM_BUILD_CHECK_HERMITIAN if check_hermitian else 0))

    def operator(self, ham, op):
        """tbpm_build_operator of an operator given as a lattice-like CSR (n, row_ptr, col, val)."""
        return tbpm_build_operator(self.handle, ham, op.n, op.row_ptr, op.col, op.val)

    def close(self) -> None:
        if self.handle:
            tbpm_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
