"""The paper's mass-solve experiments on the GPU path, against the iteration
counts its Tables h1_mass_solve, hcurl_mass_solve and hdiv_mass_solve print
(tests/golden/paper_mass_solve_tables.json; about 1e6 DOFs, random
right-hand side, u_0 = 0, relative residual 1e-10, cap 5000).

What is compared, and why with a tolerance: the paper's meshes, right-hand
side and power-iteration start are not specified exactly (its meshes are
Firedrake's; here: unjittered Kuhn meshes with the DOF count closest to 1e6),
so counts agree to a few percent, not exactly.
* CG iterations with BRAS, every family and degree:  |ours - paper| <= max(2, 8%).
* CG iterations with the diagonal, where the degree-of-freedom variant is
  pinned (Lagrange and Bernstein; degree 1 of the vector families except 3D
  BDM_1): the same bound.  Elsewhere the paper does not state its moment
  variant and the diagonal of M depends on it (parity unpinned): not
  asserted.  BRAS does not depend on it (entity-wise basis changes leave its
  spectrum unchanged).
* Fixed-point updates (weights from the power iteration): |ours - paper| <=
  max(3, 15%) under the same pinning rule; an entry the paper marks as capped
  at 5000 must reach the cap here as well.
"""
import json
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_mass_solve_tables.json")
FAMILIES = ("P", "B", "N1curl", "RT", "N2curl", "BDM")
CASES = [c for c in json.load(open(GOLDEN))["cases"] if c["family"] in FAMILIES]


def ids(c):
    return "%s%d-%dd" % (c["family"], c["degree"], c["dim"])


def pinned_diag(c):
    # degree 1 has one moment space per entity whose orthonormal basis is unique
    # up to signs, except the P_1 face moments of 3D BDM_1
    return c["family"] in ("P", "B") or (c["degree"] == 1 and not (c["family"] == "BDM" and c["dim"] == 3))


def close(ours, paper, rel, floor):
    return abs(ours - paper) <= max(floor, rel * paper)


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_iteration_counts_match_paper(case):
    from paper_2607_12138_amd import tables
    print("paper table case %s (%s)" % (ids(case), case["cite"]), flush=True)
    sys.stdout.flush()
    r = tables.run_case(case["family"], case["dim"], case["degree"])
    print(json.dumps(r), flush=True)
    assert max(r["cg_relres"]) <= 1e-9                      # true residual at exit
    sides = (0, 1) if pinned_diag(case) else (1,)
    for s in sides:
        assert close(r["cg_its"][s], case["cg_its"][s], 0.08, 2), ("cg", s, r["cg_its"], case["cg_its"])
        if case["fp_capped"][s]:
            assert r["fp_status"][s] != 0 and r["fp_its"][s] == 5000
        else:
            assert r["fp_status"][s] == 0
            assert close(r["fp_its"][s], case["fp_its"][s], 0.15, 3), ("fp", s, r["fp_its"], case["fp_its"])
    # BRAS: lambda_min >= 1 makes 2/(1 + lambda_max) a convergent weight, and the
    # Chebyshev iteration on [1, 1.02 lambda_max] needs no more updates than
    # the fixed point
    assert r["lambda_max"][1] >= 1.0
    assert r["cheb_bras_its"] <= r["fp_its"][1]
