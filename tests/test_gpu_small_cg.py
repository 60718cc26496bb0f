"""The single work-group PCG solver of small problems (Section 3's iteration
in one kernel, CG vectors in LDS) against the oracle's PCG and against the
multi-pass solver: iteration counts, solutions, every preconditioner, the
maxit / zero right-hand side / warm-start outcomes, reproducibility, and the
problems that must take the multi-pass path."""
import sys

import numpy as np
import pytest

from oracle import fe as ofe, mesh as omesh, assembly as oasm, pcg as opcg
import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-10

CASES = [
    # family, dim, degree, N, jitter, density
    ("P", 2, 1, 32, 0.0, False),   # n = 1089: the 32^2 P1 workload
    ("P", 2, 1, 9, 0.2, True),     # lognormal element densities
    ("P", 2, 3, 7, 0.2, False),    # n_loc 10
    ("P", 3, 1, 8, 0.2, False),    # n = 729
    ("P", 3, 2, 5, 0.2, True),     # n = 1331, n_loc 10
    ("B", 2, 4, 5, 0.2, False),    # Bernstein, n_loc 15
    ("P", 3, 4, 2, 0.0, False),    # n_loc 35
]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def ids(c):
    return "%s%d-%dd-N%d%s" % (c[0], c[2], c[1], c[3], "-rho" if c[5] else "")


def build(case, seed=5):
    from paper_2607_12138_amd.problem import MassProblem
    family, dim, deg, N, jit, dens = case
    coords, cells = omesh.structured_mesh(dim, N, jitter=jit, seed=seed)
    rho = workloads.density(len(cells), 77) if dens else None
    orc = oasm.Problem(ofe.reference_element(family, dim, deg), coords, cells, rho=rho)
    say("setup %s" % (case,))
    gpu = MassProblem(family, dim, deg, N, jitter=jit, seed=seed, rho=rho)
    assert gpu.n == orc.n
    return orc, gpu


def solve(gpu, b, pc, small, rtol=TOL, maxit=5000, x0=None):
    from paper_2607_12138_amd import _lib as L
    L.bras_set_option(gpu.h, L.OPT_SMALL_CG, 1 if small else 0)
    x, st, its, rel = gpu.solve(b, pc, rtol=rtol, maxit=maxit, x0=x0)
    assert gpu.info("solve_path") == (1 if small else 0)
    return x.cpu().numpy(), st, int(its[0]), float(rel[0])


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_small_solver_matches_oracle_and_multipass(case):
    import torch
    from paper_2607_12138_amd import _lib as L
    orc, gpu = build(case)
    b = workloads.rhs(orc.n, 1, 3)
    bt = torch.from_numpy(b).cuda()
    Cs = {"none": None, "jacobi": opcg.jacobi(orc.diag), "bras": orc.B.dot}
    for pc in ("none", "jacobi", "bras"):
        say("  %s" % pc)
        xo, ito, ok, _ = opcg.pcg(orc.M, b, Cs[pc], tol=TOL)
        assert ok
        xs, sts, its_s, rel_s = solve(gpu, bt, pc, True)
        xm, stm, its_m, rel_m = solve(gpu, bt, pc, False)
        say("    iterations oracle %d, one work-group %d, multi-pass %d" % (ito, its_s, its_m))
        assert sts == L.BRAS_OK and stm == L.BRAS_OK
        # counts agree up to rounding; long unpreconditioned runs on the
        # density meshes drift by a few iterations between any two orders
        slack = max(1, int(0.02 * ito))
        assert abs(its_s - ito) <= slack and abs(its_s - its_m) <= slack
        assert rel_s <= 1.5 * TOL
        # true residual reported = the one recomputed here from the returned x
        nb = np.linalg.norm(b)
        assert abs(np.linalg.norm(b - orc.M @ xs) / nb - rel_s) <= 1e-3 * TOL + 1e-14
        # the solutions solve the same system to the tolerance: M (x - x') is
        # bounded by the two residuals whatever the conditioning
        for other in (xo, xm):
            assert np.linalg.norm(orc.M @ (xs - other)) <= 4 * TOL * nb
    gpu.close()


def test_small_solver_maxit_and_iterates():
    """With maxit = 4 both paths stop after four products M p (ENOCONV) at the
    same iterate, which is also the oracle's fourth iterate."""
    import torch
    from paper_2607_12138_amd import _lib as L
    orc, gpu = build(("P", 2, 2, 10, 0.2, True))
    b = workloads.rhs(orc.n, 1, 9)
    bt = torch.from_numpy(b).cuda()
    xo, ito, ok, _ = opcg.pcg(orc.M, b, orc.B.dot, tol=TOL, maxit=4)
    assert not ok and ito == 4
    xs, sts, its_s, _ = solve(gpu, bt, "bras", True, maxit=4)
    xm, stm, its_m, _ = solve(gpu, bt, "bras", False, maxit=4)
    assert sts == stm == L.BRAS_ENOCONV and its_s == its_m == 4
    assert np.linalg.norm(xs - xm) <= 1e-12 * np.linalg.norm(xm)
    assert np.linalg.norm(xs - xo) <= 1e-11 * np.linalg.norm(xo)
    gpu.close()


def test_small_solver_zero_rhs_and_warm_start():
    import torch
    from paper_2607_12138_amd import _lib as L
    orc, gpu = build(("P", 2, 1, 12, 0.2, False))
    zero = torch.zeros(orc.n, dtype=torch.float64, device="cuda")
    x, st, its, rel = solve(gpu, zero, "bras", True)
    assert st == L.BRAS_OK and its == 0 and rel == 0.0 and not x.any()
    # warm start from a loose solve: x_d is read as x_0 and overwritten
    b = workloads.rhs(orc.n, 1, 4)
    bt = torch.from_numpy(b).cuda()
    x0 = gpu.solve(bt, "bras", rtol=1e-3)[0]
    r0 = np.linalg.norm(b - orc.M @ x0.cpu().numpy())
    xo, ito, ok, _ = opcg.pcg(orc.M, b, orc.B.dot, x0=x0.cpu().numpy(), tol=TOL)
    xs, sts, its_s, rel_s = solve(gpu, bt, "bras", True, x0=x0)
    xm, stm, its_m, rel_m = solve(gpu, bt, "bras", False, x0=x0)
    assert sts == stm == L.BRAS_OK and abs(its_s - ito) <= 1 and abs(its_s - its_m) <= 1
    # relres is relative to the warm start's residual
    assert abs(rel_s * r0 - np.linalg.norm(b - orc.M @ xs)) <= 1e-2 * TOL * r0 + 1e-14 * np.linalg.norm(b)
    assert np.linalg.norm(xs - xo) <= 1e-8 * np.linalg.norm(xo)
    gpu.close()


def test_small_solver_is_reproducible():
    import torch
    orc, gpu = build(("P", 3, 2, 5, 0.2, True))
    bt = torch.from_numpy(workloads.rhs(orc.n, 1, 6)).cuda()
    a = solve(gpu, bt, "bras", True)
    b = solve(gpu, bt, "bras", True)
    assert np.array_equal(a[0], b[0]) and a[2] == b[2] and a[3] == b[3]
    gpu.close()


def test_problems_outside_the_small_solver_use_multipass():
    import torch
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import MassProblem
    cases = [
        (dict(family="P", dim=2, degree=1, N=46), 1, "f64", 5000),     # n = 2209 > 2048
        (dict(family="P", dim=3, degree=1, N=10), 1, "f64", 5000),     # 6000 elements > 3 x 1024
        (dict(family="P", dim=2, degree=2, N=30), 1, "f64", 5000),     # LDS: 16 n + 10 n_br > 160000
        (dict(family="P", dim=2, degree=1, N=8), 2, "f64", 5000),      # two columns
        (dict(family="RT", dim=2, degree=1, N=8), 1, "f32", 5000),     # FP32 inverses
        (dict(family="N1curl", dim=2, degree=1, N=8), 1, "f64", 5000),  # metric form
        (dict(family="P", dim=2, degree=1, N=8), 1, "f64", 200000),    # maxit above the cap
    ]
    for kw, R, prec, maxit in cases:
        say("fallback %s R=%d %s maxit=%d" % (kw, R, prec, maxit))
        gpu = MassProblem(prec=prec, max_rhs=R, jitter=0.1, seed=2, **kw)
        b = workloads.rhs(gpu.n, R, 8)
        bt = torch.from_numpy(b).cuda()
        x, st, its, rel = gpu.solve(bt, "bras", rtol=1e-8, maxit=maxit)
        assert st == L.BRAS_OK and gpu.info("solve_path") == 0
        gpu.close()
    gpu = MassProblem("P", 2, 1, 8)
    with pytest.raises(L.BrasError) as e:
        L.bras_set_option(gpu.h, L.OPT_SMALL_CG, 2)
    assert e.value.code == L.BRAS_EINVAL
    gpu.close()


def stationary(gpu, kind, b, pc, small, **kw):
    from paper_2607_12138_amd import _lib as L
    L.bras_set_option(gpu.h, L.OPT_SMALL_CG, 1 if small else 0)
    fn = gpu.fixed_point if kind == "fp" else gpu.chebyshev
    x, st, its, rel = fn(b, pc, **kw)
    assert gpu.info("solve_path") == (1 if small else 0)
    return x.cpu().numpy(), st, int(its[0]), float(rel[0])


@pytest.mark.parametrize("case", [CASES[0], CASES[1], CASES[4], CASES[6]], ids=ids)
def test_small_stationary_matches_oracle_and_multipass(case):
    """Damped fixed point (BRAS and Jacobi weights from the power iteration)
    and Chebyshev with BRAS on [1, 1.02 lambda_max] (Section 3)."""
    import torch
    from oracle import stationary as ost
    from paper_2607_12138_amd import _lib as L
    orc, gpu = build(case)
    f = workloads.rhs(orc.n, 1, 12)
    ft = torch.from_numpy(f).cuda()
    nf = np.linalg.norm(f)
    v0 = workloads.vector(orc.n, 7)
    runs = []
    for pc, C in (("bras", orc.B.dot), ("jacobi", opcg.jacobi(orc.diag))):
        lam = ost.power_lambda_max(orc.M, C, v0, iters=50)
        om = 2.0 / (1.0 + lam) if pc == "bras" else 1.0 / lam
        runs.append(("fp", pc, dict(omega=om), ost.fixed_point(orc.M, f, C, om, tol=TOL)))
        if pc == "bras":
            runs.append(("cheb", pc, dict(lmin=1.0, lmax=1.02 * lam),
                         ost.chebyshev(orc.M, f, C, 1.0, 1.02 * lam, tol=TOL)))
    for kind, pc, kw, (xo, ito, ok, _) in runs:
        assert ok
        xs, sts, its_s, rel_s = stationary(gpu, kind, ft, pc, True, rtol=TOL, **kw)
        xm, stm, its_m, rel_m = stationary(gpu, kind, ft, pc, False, rtol=TOL, **kw)
        say("  %s %s: oracle %d, one work-group %d, multi-pass %d" % (kind, pc, ito, its_s, its_m))
        assert sts == stm == L.BRAS_OK
        assert abs(its_s - ito) <= 1 and abs(its_s - its_m) <= 1
        # relres is the residual of the returned iterate
        assert abs(np.linalg.norm(f - orc.M @ xs) / nf - rel_s) <= 1e-3 * TOL + 1e-14
        for other in (xo, xm):
            assert np.linalg.norm(orc.M @ (xs - other)) <= 4 * TOL * nf
    gpu.close()


def test_small_stationary_maxit_and_zero_rhs():
    import torch
    from oracle import stationary as ost
    from paper_2607_12138_amd import _lib as L
    orc, gpu = build(("P", 2, 2, 10, 0.2, True))
    f = workloads.rhs(orc.n, 1, 13)
    ft = torch.from_numpy(f).cuda()
    lam = ost.power_lambda_max(orc.M, orc.B.dot, workloads.vector(orc.n, 7), iters=50)
    om = 2.0 / (1.0 + lam)
    xo, ito, ok, _ = ost.fixed_point(orc.M, f, orc.B.dot, om, tol=TOL, maxit=3)
    assert not ok and ito == 3
    xs, sts, its_s, _ = stationary(gpu, "fp", ft, "bras", True, omega=om, rtol=TOL, maxit=3)
    xm, stm, its_m, _ = stationary(gpu, "fp", ft, "bras", False, omega=om, rtol=TOL, maxit=3)
    assert sts == stm == L.BRAS_ENOCONV and its_s == its_m == 3
    assert np.linalg.norm(xs - xm) <= 1e-13 * np.linalg.norm(xm)
    assert np.linalg.norm(xs - xo) <= 1e-12 * np.linalg.norm(xo)
    zero = torch.zeros(orc.n, dtype=torch.float64, device="cuda")
    x, st, its, rel = stationary(gpu, "cheb", zero, "bras", True, lmin=1.0, lmax=1.02 * lam, rtol=TOL)
    assert st == L.BRAS_OK and its == 0 and rel == 0.0 and not x.any()
    gpu.close()
