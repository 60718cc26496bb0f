"""The rotated-stretch study of Section 3 (eq. rot_stretch_map, Cor.
bras_piola_metric_contrast) run through libbras on one GPU.

2D BDM_p on the unit-square Kuhn mesh mapped by x -> c + R S R^T (x - c)
(det 1, singular values r and 1/r, so the H(div) metric contrast relative to
the unmapped mesh is r^4).  Per (p, r): the power-iteration lambda_max of
Mbras^-1 M (its lambda_min is 1, so this is kappa-hat of BRAS) and of
diag(M)^-1 M, and the CG iteration counts of both preconditioners
(relative residual 1e-10).  The mesh has about `--dofs` conforming DOFs
(the study uses about 5e3).

    python -m paper_2607_12138_amd.stretch [--degrees 1,3,5,7] [--r 1,3,5,7] [--dofs 5000]
"""
import argparse
import json
import sys

from . import tables

SEED = 0x260712138 + 0x57E7C


def run_case(degree, r, dofs=5000, iters=300):
    import torch
    import workloads
    from .problem import MassProblem

    N = tables.mesh_for("BDM", 2, degree, dofs)
    mp = MassProblem("BDM", 2, degree, N, coord_map=lambda x: workloads.rotated_stretch(x, r))
    v0 = workloads.vector(mp.n, SEED + degree)
    b = torch.from_numpy(workloads.rhs(mp.n, 1, SEED + 100 + degree)).to(mp.device)
    out = {"family": "BDM", "dim": 2, "degree": degree, "r": r, "N": N, "n": mp.n, "n_loc": mp.n_loc}
    out["lambda_max"] = [round(mp.lambda_max(pc, v0, iters), 6) for pc in ("jacobi", "bras")]
    out["cg_its"] = [int(mp.solve(b, pc, 1e-10, 5000)[2][0]) for pc in ("jacobi", "bras")]
    mp.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--degrees", default="1,3,5,7")
    ap.add_argument("--r", default="1,3,5,7")
    ap.add_argument("--dofs", type=int, default=5000)
    a = ap.parse_args(argv)
    for p in map(int, a.degrees.split(",")):
        for r in map(float, a.r.split(",")):
            print(json.dumps(run_case(p, r, a.dofs)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
