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


def test_iteration_bytes_cover_both_kernels_and_the_vectors():
    # 32^3 p = 3 elasticity: the two streaming kernels plus the CG vector
    # passes (10 FP64 vectors of n), the block outputs read back by the pull
    # and its node -> block map
    n_nodes = 97 ** 3
    n = 3 * n_nodes
    info = {"n_dofs": n, "bsr_dim": 3, "nnzb": 111_284_641, "lattice_columns": True}
    spmv, schwarz = bench.algorithmic_bytes(info, m=192, n_blocks=32_768, nn=64)
    it = bench.iteration_bytes(info, m=192, n_blocks=32_768, nn=64)
    pull = 32_768 * 192 * 8 + 32_768 * 64 * 4 + (n_nodes + 1) * 4
    assert it == spmv + schwarz + pull + 12 * n * 8
    # below the 18.49 GB of a layout that stores every inverse in full and
    # reads the block columns: the wrapped-diagonal half and the lattice
    # columns save 5.2 GB
    assert 13.0e9 < it < 13.5e9
