"""Host checks of bench.py's accounting (no GPU): the algorithmic bytes per
launch of the dominant kernel, for both series evaluations, match the counts
written out by hand from the kernels' reads and writes, and the run refuses
more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

N = 33554432                    # graphene 4096 x 4096
NNZ = 134217728


def test_graphene_c128_patch_pairs():
    info = {"format": 3, "ell_w": 4, "nnz": NNZ}
    h = 4 * N * (16 + 2)                                     # w slots of (complex128 value, 2-byte local column)
    assert bench.algorithmic_bytes_per_launch(info, N, 1, "c128") == (h + 6 * 16 * N, h, 2)
    assert bench.algorithmic_bytes_per_launch(info, N, 1, "c128", True) == (h + 5 * 16 * N, h, 2)
    assert h + 6 * 16 * N == 5637144576                     # the headline kernel's figure


def test_single_terms_ell_and_blocks():
    info = {"format": 1, "ell_w": 4, "nnz": NNZ}
    h = 4 * N * 20
    assert bench.algorithmic_bytes_per_launch(info, N, 1, "c128") == (h + 5 * 16 * N, h, 1)
    assert bench.algorithmic_bytes_per_launch(info, N, 1, "c128", True) == (h + 4 * 16 * N, h, 1)
    # patch format with a block of 16 complex64 vectors: the staged SpMM (2-byte local
    # columns four to an 8-byte word: 16 bytes for 5 slots)
    n, B = 16777216, 16
    info = {"format": 3, "ell_w": 5, "nnz": 75497472}
    h = n * (5 * 8 + 16)
    assert bench.algorithmic_bytes_per_launch(info, n, B, "c64") == (h + 5 * 8 * n * B, h, 1)
    assert bench.algorithmic_bytes_per_launch(info, n, B, "c64", True) == (h + 4 * 8 * n * B, h, 1)


def test_complex64_block_pairs():
    # 3rd-neighbour honeycomb, block of 8 that the library pairs: H once (2-byte columns and
    # one-byte indices, 12 slots) and six vector passes for two terms; Clenshaw stays single
    n, B = 96_000_000, 8
    info = {"format": 3, "ell_w": 12, "nnz": 12 * n, "table_used": True, "table_diag": 0, "block_pairs": True}
    h = n * (12 * 2 + 12)
    assert bench.algorithmic_bytes_per_launch(info, n, B, "c64") == (h + 6 * 8 * n * B, h, 2)
    assert bench.algorithmic_bytes_per_launch(info, n, B, "c64", True) == (h + 4 * 8 * n * B, h, 1)
    assert "6 vector passes for two terms" in bench.bytes_model_text(info, B, 2, False, "propagate")


def test_value_table_bytes():
    # graphene with on-site disorder: one index word (4 slots) and the real part of the row's diagonal
    info = {"format": 3, "ell_w": 4, "nnz": NNZ, "table_used": True, "table_diag": 2}
    h = N * (4 * 2 + 4 + 8)
    assert bench.algorithmic_bytes_per_launch(info, N, 1, "c128") == (h + 6 * 16 * N, h, 2)
    # 3rd-neighbour honeycomb, no on-site term: 12 slots in 3 index words, 2-byte columns (staged SpMM)
    n, B = 96_000_000, 8
    info = {"format": 3, "ell_w": 12, "nnz": 12 * n, "table_used": True, "table_diag": 0}
    h = n * (12 * 2 + 12)
    assert bench.algorithmic_bytes_per_launch(info, n, B, "c64") == (h + 5 * 8 * n * B, h, 1)
    # other blocks on the patch format read the values
    assert bench.algorithmic_bytes_per_launch(info, n, 4, "c64")[1] == 12 * n * 12
    # AB bilayer with disorder: 5 slots in 2 words + the diagonal's real part (complex64)
    n = 16777216
    info = {"format": 3, "ell_w": 5, "nnz": 5 * n, "table_used": True, "table_diag": 2}
    assert bench.algorithmic_bytes_per_launch(info, n, 16, "c64")[1] == n * (16 + 8 + 4)
    info["table_diag"] = 1
    assert bench.algorithmic_bytes_per_launch(info, n, 16, "c64")[1] == n * (16 + 8 + 8)
    assert "value table" in bench.bytes_model_text(info, 16, 1, False, "propagate")
    # without the table: every value
    info["table_used"] = False
    assert bench.algorithmic_bytes_per_launch(info, n, 16, "c64")[1] == n * (16 + 5 * 8)


def test_csr_row_pointer_bytes():
    info = {"format": 0, "ell_w": 0, "nnz": 1000}
    assert bench.algorithmic_bytes_per_launch(info, 100, 1, "c128")[1] == 1000 * 20 + 101 * 4


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_forward_recurrence_step_bytes_by_hand():
    """(M-1) products streaming H plus (5M-6) vector passes per step; with M = 20
    for graphene 4096^2 in complex128 (ELL width 4): 19 H + 94 vector passes."""
    h = 4 * N * 20
    assert 19 * h + (5 * 20 - 6) * 16 * N == 19 * 2684354560 + 94 * 536870912


def test_traffic_summary_checks_series_and_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    f = tmp_path / "profiles" / "traffic_mid_term_w.txt"
    f.write_text(f"# header\nseries: forward\nhbm_bytes_per_launch: 123\nsource_sha256: {bench.traffic_source_hash()}\n")
    assert bench.read_traffic("mid_term", "w", "forward") == 123.0
    assert bench.read_traffic("mid_term", "w", "clenshaw") is None
    f.write_text("series: forward\nhbm_bytes_per_launch: 123\nsource_sha256: 00\n")
    assert bench.read_traffic("mid_term", "w", "forward") is None


def test_host_cpu_description():
    h = bench.host_cpu()
    assert h["logical_cpus"] >= 1 and h["cpus_usable_by_process"] >= 1
    assert h["physical_cores"] is None or 1 <= h["physical_cores"] <= h["logical_cpus"]
