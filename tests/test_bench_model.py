"""The byte model bench.py divides by the measured kernel times (CPU only):
the algorithmic bytes of one SpMV and one block-product launch, written out
for the two FP64 workloads from their sizes."""
import importlib.util
import os

import pytest

_spec = importlib.util.spec_from_file_location(
    "bench_module", os.path.join(os.path.dirname(__file__), "..", "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)


def test_elasticity_workload_bytes():
    # 32^3 cells, p = 3, 3 components: 97^3 nodes, 481^3 / 9 ... 3x3 blocks
    n_nodes = 97 ** 3
    info = {"n_dofs": 3 * n_nodes, "bsr_dim": 3, "nnzb": 111_284_641, "lattice_columns": True}
    spmv, schwarz = bench.algorithmic_bytes(info, m=192, n_blocks=32_768, nn=64)
    assert spmv == 111_284_641 * 72 + (n_nodes + 1) * 4 + 2 * 3 * n_nodes * 8
    assert spmv == pytest.approx(8.060e9, rel=1e-3)
    assert schwarz == 32_768 * 97 * 192 * 8 + 32_768 * 64 * 4 + 2 * 3 * n_nodes * 8 + 32_768 * 192 * 8
    # with stored columns the SpMV also reads 4 bytes per block
    info["lattice_columns"] = False
    spmv_cols, _ = bench.algorithmic_bytes(info, m=192, n_blocks=32_768, nn=64)
    assert spmv_cols - spmv == 111_284_641 * 4


def test_poisson_workload_bytes():
    # 64^3 cells, p = 2, scalar: 129^3 unknowns, 513^3 stored entries
    n = 129 ** 3
    info = {"n_dofs": n, "bsr_dim": 1, "nnzb": 513 ** 3, "lattice_columns": True}
    spmv, schwarz = bench.algorithmic_bytes(info, m=27, n_blocks=64 ** 3, nn=27)
    assert spmv == 513 ** 3 * 8 + (n + 1) * 4 + 2 * n * 8
    assert spmv == pytest.approx(1.123e9, rel=1e-3)
    assert schwarz == 64 ** 3 * 14 * 27 * 8 + 64 ** 3 * 27 * 4 + 2 * n * 8 + 64 ** 3 * 27 * 8


def test_shared_copies_bytes():
    # the same elasticity workload with the kept copies it has at set-up:
    # 103,041,504 kept row values (one 8-byte offset per block row) and
    # 8,817 kept inverses (one 8-byte offset per block)
    n_nodes = 97 ** 3
    info = {"n_dofs": 3 * n_nodes, "bsr_dim": 3, "nnzb": 111_284_641, "lattice_columns": True,
            "shared_values": 103_041_504}
    spmv, schwarz = bench.algorithmic_bytes(info, m=192, n_blocks=32_768, nn=64,
                                            distinct_blocks=8_817)
    assert spmv == (103_041_504 * 8 + n_nodes * 8 + (n_nodes + 1) * 4
                    + 2 * 3 * n_nodes * 8)
    assert spmv == pytest.approx(0.879e9, rel=1e-3)
    assert schwarz == (8_817 * 97 * 192 * 8 + 32_768 * (64 * 4 + 8) + 2 * 3 * n_nodes * 8
                       + 32_768 * 192 * 8)
    assert schwarz == pytest.approx(1.416e9, rel=1e-3)
