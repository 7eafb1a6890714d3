"""Writes small_alpha_cube.json: the oracle's Schwarz-PCG on a 6^3-cell,
p = 3 elasticity cube whose large spherical void holds eight cells
entirely, at fictitious stiffness alpha = 1e-16 and 1e-12, with the
stabilised pseudo-inverses (S, Sec. 3.2 Eqs. 9-11) and the plain inverses
(S*), and at 1e-12 with S after removing the functions of the void cells
(the paper's preprocessing, Sec. 5.2), stopped at ||z|| / ||z_0|| <= 1e-10
(Eq. 12) or 20,000 iterations.
Only the oracle is called.  Run from the repository root:
    python tests/golden/make_small_alpha_cube.py
(about 8 minutes on one core)."""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "..", ".."))
import fcgen  # noqa: E402
from oracle import assemble as ASM  # noqa: E402
from oracle import pcg as PCG  # noqa: E402
from oracle import schwarz as SCH  # noqa: E402

SHAPES = [{"centre": [0.5, 0.52, 0.48], "semi": [0.33, 0.33, 0.33]},
          {"centre": [0.2, 0.25, 0.7], "semi": [0.12, 0.12, 0.12]}]
NAMES = {PCG.OK: "OK", PCG.NOTCONV: "E_NOTCONV", PCG.BREAKDOWN: "E_BREAKDOWN"}


def desc(alpha, discard=False):
    return fcgen.custom(3, 6, 3, pde="elasticity", alpha=alpha, shapes=SHAPES, clamp_zmin=True,
                        discard_fictitious=discard)


def main():
    out = {"shapes": SHAPES, "n": 6, "p": 3, "tol": 1e-10, "maxit": 20000, "runs": []}
    for alpha, discard in ((1e-16, False), (1e-12, False), (1e-12, True)):
        s = ASM.assemble(desc(alpha, discard))
        A, b = s["A"], s["b"]
        blocks = SCH.select_blocks(s["elem_dofs"], s["eta"], 1.0)
        dropped = 0
        for B in blocks:
            lam = np.linalg.eigvalsh(SCH.extract_submatrix(A, B))
            dropped += int((lam <= 1e-13 * lam.max()).sum())
        for stab in ((True,) if discard else (True, False)):
            S, _ = SCH.compute_preconditioner(A, blocks, stabilize=stab)
            x, info = PCG.pcg(A, b, S, tol=1e-10, maxit=20000, stop="precond")
            finite = bool(np.isfinite(x).all())
            res = float(np.linalg.norm(b - A @ x) / np.linalg.norm(b)) if finite else None
            rec = {"alpha": alpha, "discard_fictitious": discard, "stabilize": stab,
                   "iters": int(info["iters"]),
                   "status": NAMES.get(info["status"], "E_NAN"), "rel_res_true": res,
                   "rel_res_prec": float(info["prec"][-1]),
                   "dropped": dropped if stab else 0,
                   "eta_zero_cells": int((s["eta"] == 0).sum())}
            print(rec, flush=True)
            out["runs"].append(rec)
    path = os.path.join(os.path.dirname(__file__), "small_alpha_cube.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
