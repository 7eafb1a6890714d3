"""The oracle's element-by-element operators against its assembled matrices.

A = sum_e R_e^T K_e R_e and S = sum_B R_B^T P_B R_B (+ Algorithm 1's
diagonal scaling), applied by gathering, multiplying and adding back
(oracle/ebe.py), must equal the products with the globally assembled A
(COO assembly with the clamped rows removed) and S (Algorithm 1's sparse
sum) to rounding: on a clamped elasticity cube with every cell a block, and
on a Poisson square where only cut cells are blocks (eta_bar = 0.5), so
Algorithm 1's diagonal scaling covers the functions of the other cells."""
import numpy as np
import pytest

import fcgen
from oracle import assemble, ebe, schwarz


def _cases():
    return {
        "elasticity": fcgen.porous_elasticity_3d(seed=3, n=3, p=2, n_voids=2),
        "poisson": fcgen.custom(2, 6, 2, "poisson", 1e-10,
                                shapes=[{"centre": (0.5, 0.5), "semi": (0.3, 0.3)}],
                                domain="voids"),
    }


ETA_BAR = {"elasticity": 1.0, "poisson": 0.5}


@pytest.mark.parametrize("name", ["elasticity", "poisson"])
def test_element_operators_equal_assembled(name):
    desc = _cases()[name]
    s = assemble.assemble(desc, keep_elements=True)
    A, n = s["A"], s["A"].shape[0]
    rng = np.random.default_rng(0)
    v = rng.standard_normal(n)
    Aop = ebe.ElementOperator(s["elem_dofs"], s["Ke"], n, clamped=assemble.clamped_dofs(desc))
    ref = A @ v
    assert np.abs(Aop @ v - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.allclose(Aop.diagonal(), A.diagonal(), rtol=1e-13, atol=0)
    blocks = schwarz.select_blocks(s["elem_dofs"], s["eta"], ETA_BAR[name])
    S, fall = schwarz.compute_preconditioner(A, blocks)
    P = np.array([schwarz.pseudo_inverse(schwarz.extract_submatrix(A, B)) for B in blocks])
    extra = np.zeros(n)
    extra[fall] = 1.0 / A.diagonal()[fall]
    Sop = ebe.ElementOperator(np.array(blocks), P, n, diag_extra=extra)
    ref = S @ v
    assert np.abs(Sop @ v - ref).max() <= 1e-11 * np.abs(ref).max()
    if name == "poisson":
        assert fall.size > 0   # the fallback diagonal is exercised
