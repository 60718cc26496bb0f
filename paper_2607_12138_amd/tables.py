"""The paper's mass-solve experiments (Section 3; Tables h1_mass_solve,
hcurl_mass_solve, hdiv_mass_solve; all six element families) run through
libbras on one GPU.

For each element family, dimension and degree the conforming system has
about 1e6 DOFs on an unjittered Kuhn mesh of the unit square / cube; the
right-hand side is U[-1, 1], u_0 = 0, every solver stops at
||r_k|| / ||r_0|| <= 1e-10 or after 5000 iterations.  Reported per case, as
[diag, BRAS] pairs: CG iterations and times, power-iteration lambda_max,
damped fixed-point updates and times with the weights 1/lambda_max (diag)
and 2/(1 + lambda_max) (BRAS), plus the BRAS Chebyshev iteration on
[1, 1.02 lambda_max].  Times exclude set-up and the lambda_max estimate, as
in the paper.

    python -m paper_2607_12138_amd.tables [--families P,B] [--dims 3] [--degrees 1,4]
"""
import argparse
import json
import sys
import time

from . import _lib as L

TOL = 1e-10
MAXIT = 5000
TARGET_DOFS = 1_000_000
POWER_ITERS = 200     # power-iteration steps for lambda_max (the paper does not state a count)
SEED = 0x260712138 + 0x7AB1E
FAMILIES = ("P", "B", "N1curl", "RT", "N2curl", "BDM")


def entity_counts(dim, N):
    """Vertices, edges, (faces,) cells of the Kuhn mesh with N cells per side."""
    if dim == 2:
        return ((N + 1) ** 2, 3 * N * N + 2 * N, 2 * N * N)
    return ((N + 1) ** 3, 7 * N ** 3 + 9 * N ** 2 + 3 * N, 12 * N ** 3 + 6 * N ** 2, 6 * N ** 3)


def dof_count(family, dim, degree, N):
    _, per = L.bras_element_info(L.FAMILY[family], dim, degree)
    return sum(a * b for a, b in zip(per, entity_counts(dim, N)))


def mesh_for(family, dim, degree, target=TARGET_DOFS):
    """The N whose DOF count is closest to `target`."""
    best = None
    for N in range(1, 2001):
        n = dof_count(family, dim, degree, N)
        if best is None or abs(n - target) < abs(best[1] - target):
            best = (N, n)
        if n > target:
            break
    return best[0]


def case_seed(family, dim, degree):
    return SEED + 64 * FAMILIES.index(family) + 8 * dim + degree


def _timed(sync, fn):
    sync()
    t0 = time.perf_counter()
    out = fn()
    sync()
    return out, 1e3 * (time.perf_counter() - t0)


def run_case(family, dim, degree, N=None, stationary=True):
    import torch
    import workloads
    from .problem import MassProblem

    N = mesh_for(family, dim, degree) if N is None else N
    seed = case_seed(family, dim, degree)
    mp = MassProblem(family, dim, degree, N, jitter=0.0, seed=seed, prec="f64")
    sync = torch.cuda.synchronize
    b = torch.from_numpy(workloads.rhs(mp.n, 1, seed)).to(mp.device)
    out = {"family": family, "dim": dim, "degree": degree, "N": N, "n": mp.n, "E": mp.E, "n_loc": mp.n_loc}
    cg_its, cg_ms, cg_rel = [], [], []
    for pc in ("jacobi", "bras"):
        mp.solve(b, pc, TOL, MAXIT)                          # warm-up (graph capture)
        (x, st, its, rel), ms = _timed(sync, lambda: mp.solve(b, pc, TOL, MAXIT))
        cg_its.append(int(its[0]))
        cg_ms.append(round(ms, 3))
        cg_rel.append(float(rel[0]))
    out.update(cg_its=cg_its, cg_ms=cg_ms, cg_relres=cg_rel)
    if stationary:
        v0 = workloads.vector(mp.n, seed + 1)
        lam = [mp.lambda_max(pc, v0, POWER_ITERS) for pc in ("jacobi", "bras")]
        om = [1.0 / lam[0], 2.0 / (1.0 + lam[1])]
        fp_its, fp_ms, fp_st = [], [], []
        for pc, w in zip(("jacobi", "bras"), om):
            (x, st, its, rel), ms = _timed(sync, lambda: mp.fixed_point(b, pc, w, TOL, MAXIT))
            fp_its.append(int(its[0]))
            fp_ms.append(round(ms, 3))
            fp_st.append(int(st))
        (x, st, its, rel), ms = _timed(sync, lambda: mp.chebyshev(b, "bras", 1.0, 1.02 * lam[1], TOL, MAXIT))
        out.update(lambda_max=[round(v, 6) for v in lam], fp_its=fp_its, fp_ms=fp_ms, fp_status=fp_st,
                   cheb_bras_its=int(its[0]), cheb_bras_ms=round(ms, 3))
    mp.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--families", default=",".join(FAMILIES))
    ap.add_argument("--dims", default="2,3")
    ap.add_argument("--degrees", default="1,2,3,4")
    ap.add_argument("--no-stationary", action="store_true")
    a = ap.parse_args(argv)
    for fam in a.families.split(","):
        for dim in map(int, a.dims.split(",")):
            for deg in map(int, a.degrees.split(",")):
                print(json.dumps(run_case(fam, dim, deg, stationary=not a.no_stationary)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
