"""GPU parity of the eigenvalue threshold of Eq. 11 (Sec. 3.2, Eqs. 9-11;
Algorithm 1) and of z = S r element by element.

Threshold cases (tests/gpu_common.THRESHOLD_CASES): one problem per block
size the library treats differently (m = 9, 27, 64 on the eigen path in
LDS; m = 81 and 192 where the certified direct inverse fails and the
eigen-decomposition in global memory takes over), each with element blocks
whose thin slivers of material give eigenvalues far below 1e-13 of the
block's largest, and none within a factor 3 of that threshold
(tests/test_oracle_threshold.py).  So:
  * the dropped count of every block must equal the oracle's exactly;
  * every local inverse of a dropping block must have rank m - dropped
    (its nonzero eigenvalues 1/lambda_k are at least 1/lambda_max, its
    rounding noise about eps / lambda_min_kept, 4e15 / kappa apart), be
    symmetric, satisfy P A_B P = P, and differ from the oracle's
    pseudo-inverse by at most the eps * kappa that FP64 data allow.
z = S r element by element: every unknown's difference is bounded by the
per-block bound of the local inverses (sum over its blocks of tol_B ||P_B||
||r_B||, tol_B = 1e-15 m kappa_B + 1e-13); unknowns whose blocks are all
well conditioned (no eigenvalue dropped and lambda_max / lambda_min <=
1e4) must also agree to 1e-9 of (|S| |r|)_i.  (An unknown in a block that
drops eigenvalues is not such a case even when the kept ones are well
conditioned: a function that couples to the rest of its block only through
entries near 1e-16 of the block's scale, like a bubble of a cell outside
the physical domain, receives z_i from eigenvector components of that
size, which no eigensolver determines to more than absolute rounding.)
"""
import numpy as np
import pytest

import paper_1809_00828_amd as fc
from oracle import schwarz
from tests.gpu_common import (PROBLEMS, THRESHOLD_CASES, dropped_count, oracle_precond,
                              oracle_system, require_gpu, threshold_case)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


_cache = {}


def lib_case(name):
    if name not in _cache:
        d, _ = oracle_system(name)
        pb = fc.Problem.setup(d)
        _cache[name] = (pb, fc.Precond(pb))
    return _cache[name]


@pytest.mark.parametrize("name", sorted(THRESHOLD_CASES))
def test_dropped_counts_match_per_block(torch, name):
    print(f"[threshold] {name}", flush=True)
    _, s, spectra = threshold_case(name)
    pb, pc = lib_case(name)
    ref = np.array([dropped_count(lam) for lam in spectra], np.int32)
    got = pc.block_dropped()
    info = pc.info()
    m = pc.m
    print(f"[threshold] {name}: m {m}, dropped {int(ref.sum())} in "
          f"{int(np.count_nonzero(ref))} blocks, eigen-path blocks {info['n_eig_blocks']}",
          flush=True)
    np.testing.assert_array_equal(got, ref)
    assert info["n_dropped"] == int(ref.sum()) > 0
    if m > 64:
        # every dropping block failed the certificate and was eigen-decomposed
        assert info["n_eig_blocks"] >= int(np.count_nonzero(ref))


@pytest.mark.parametrize("name", sorted(THRESHOLD_CASES))
def test_pseudo_inverses_of_dropping_blocks(torch, name):
    _, s, spectra = threshold_case(name)
    pb, pc = lib_case(name)
    A = s["A"]
    m = pc.m
    eps = np.finfo(float).eps
    drops = np.array([dropped_count(lam) for lam in spectra])
    picks = list(np.nonzero(drops)[0]) + [int(np.argmin(drops))]
    for k in picks:
        B = s["elem_dofs"][k]
        AB = schwarz.extract_submatrix(A, B)
        lam = spectra[k]
        kept = lam[lam > 1e-13 * lam.max()]
        kappa = kept.max() / kept.min()
        P = pc.block_inverse(k)
        np.testing.assert_allclose(P, P.T, rtol=0, atol=1e-14 * np.abs(P).max())
        mu = np.abs(np.linalg.eigvalsh(0.5 * (P + P.T)))
        split = np.sqrt((1.0 / kept.max()) * (m * eps / kept.min()))
        assert int(np.sum(mu > split)) == m - drops[k], (k, drops[k])
        tol = 1e-15 * m * kappa + 1e-13
        ref = schwarz.pseudo_inverse(AB)
        nP = np.linalg.norm(ref)
        assert np.linalg.norm(P - ref) <= tol * nP, (k, kappa)
        assert np.linalg.norm(P @ AB @ P - P) <= 3 * tol * nP + m * eps * kappa * nP, k


def _elementwise_bound(name, r):
    """Per-unknown bound implied by the block-level tolerance, the largest
    full condition number of the blocks of every unknown (infinite for a
    block that drops eigenvalues), and (|S| |r|)."""
    _, s = oracle_system(name)
    S, _, blocks = oracle_precond(name)
    n = S.shape[0]
    bound = np.zeros(n)
    kap = np.zeros(n)
    for B in blocks:
        lam = np.linalg.eigvalsh(schwarz.extract_submatrix(s["A"], B))
        if lam.max() <= 0:
            continue
        kept = lam[lam > 1e-13 * lam.max()]
        kappa = kept.max() / kept.min()
        tol = 1e-15 * B.size * kappa + 1e-13
        bound[B] += tol * np.sqrt(np.sum(1.0 / kept ** 2)) * np.linalg.norm(r[B])
        full = kappa if kept.size == lam.size else np.inf
        kap[B] = np.maximum(kap[B], full)
    mag = abs(S) @ np.abs(r)
    return S @ r, bound, kap, mag


@pytest.mark.parametrize("name", sorted(PROBLEMS) + sorted(THRESHOLD_CASES))
def test_apply_M_elementwise(torch, name):
    print(f"[apply_M elementwise] {name}", flush=True)
    pb, pc = lib_case(name)
    r = np.random.default_rng(31).standard_normal(pb.n)
    z = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    pc.apply_M(torch.as_tensor(r, device="cuda"), z)
    torch.cuda.synchronize()
    ref, bound, kap, mag = _elementwise_bound(name, r)
    d = np.abs(z.cpu().numpy() - ref)
    assert np.all(d <= bound), (int(np.argmax(d - bound)), float(np.max(d - bound)))
    well = kap <= 1e4
    print(f"[apply_M elementwise] {name}: {int(well.sum())} of {pb.n} unknowns in "
          f"well-conditioned blocks, worst relative {float(np.max(d[well] / mag[well])) if well.any() else 0:.1e}",
          flush=True)
    if well.any():
        assert np.all(d[well] <= 1e-9 * mag[well])
