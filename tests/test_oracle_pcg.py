"""Pins for the oracle's PCG against brute force and the paper's iteration counts."""
import json
import os

import numpy as np
import pytest

from oracle import fe, mesh, assembly, pcg
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def problem(family, dim, deg, N, jitter=0.0, seed=3):
    ref = fe.reference_element(family, dim, deg)
    coords, cells = mesh.structured_mesh(dim, N, jitter=jitter, seed=seed)
    return assembly.Problem(ref, coords, cells)


@pytest.mark.parametrize("family,dim,deg,N", [("P", 3, 3, 2), ("RT", 3, 2, 2), ("N1curl", 3, 2, 2), ("P", 2, 4, 4)])
def test_pcg_matches_direct_solve(family, dim, deg, N):
    pr = problem(family, dim, deg, N, 0.2)
    b = workloads.rhs(pr.n, 1, 17)
    Md = pr.M.toarray()
    xs = np.linalg.solve(Md, b)
    cond = np.linalg.cond(Md)
    for C in (None, pcg.jacobi(pr.diag), pr.B.dot):
        x, its, ok, hist = pcg.pcg(pr.M, b, C, tol=1e-12, maxit=5000)
        assert ok
        assert np.linalg.norm(b - pr.M @ x) <= 1.01e-12 * np.linalg.norm(b) + 1e-14 * cond * np.linalg.norm(b)
        assert np.linalg.norm(x - xs) <= max(cond * 1e-11, 1e-10) * np.linalg.norm(xs)


def test_iteration_count_definition():
    pr = problem("P", 2, 2, 5, 0.2)
    b = workloads.rhs(pr.n, 1, 2)
    x, its, ok, hist = pcg.pcg(pr.M, b, pr.B.dot, tol=1e-10)
    # history holds ||r_k||/||r_0|| for k = 0..its; only the last passes the test
    assert len(hist) == its + 1 and hist[-1] <= 1e-10 and all(h > 1e-10 for h in hist[:-1])


def test_flexible_variant_agrees_with_standard():
    pr = problem("RT", 3, 2, 2, 0.2)
    b = workloads.rhs(pr.n, 1, 4)
    x1, i1, _, _ = pcg.pcg(pr.M, b, pr.B.dot, tol=1e-10)
    x2, i2, _, _ = pcg.pcg(pr.M, b, pr.B.dot, tol=1e-10, flexible=True)
    assert abs(i1 - i2) <= 1
    assert np.linalg.norm(x1 - x2) <= 1e-8 * np.linalg.norm(x1)


def test_warm_start_resumes():
    pr = problem("P", 3, 2, 2, 0.2)
    b = workloads.rhs(pr.n, 1, 6)
    xa, _, _, _ = pcg.pcg(pr.M, b, pr.B.dot, tol=1e-4)
    xb, its, ok, _ = pcg.pcg(pr.M, b, pr.B.dot, x0=xa, tol=1e-10)
    assert ok and np.linalg.norm(b - pr.M @ xb) <= 1e-10 * np.linalg.norm(b - pr.M @ xa) * 1.01


def test_cg_rate_bound_reproduces_table_counts():
    # Section 3: observed CG rates follow 2((sqrt k - 1)/(sqrt k + 1))^k closely;
    # with the printed kappa-hat 4.0 (diag, 2D P1) the bound gives the printed 22.
    assert pcg.cg_iteration_bound(4.0, 1e-10) == 22
    assert pcg.cg_iteration_bound(1.6, 1e-10) in (11, 12)


@pytest.mark.slow
@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "paper_cg_iterations.json")))["cases"],
                         ids=lambda c: c["cite"])
def test_cg_iterations_match_paper(case):
    pr = problem(case["family"], case["dim"], case["degree"], case["N"])
    assert 0.9e6 <= pr.n <= 1.1e6                 # "approximately 1e6 DOFs"
    b = workloads.rhs(pr.n, 1, 1)
    _, it_d, ok_d, _ = pcg.pcg(pr.M, b, pcg.jacobi(pr.diag), tol=1e-10)
    _, it_b, ok_b, _ = pcg.pcg(pr.M, b, pr.B.dot, tol=1e-10)
    assert ok_d and ok_b
    assert abs(it_d - case["its_diag"]) <= 1 and abs(it_b - case["its_bras"]) <= 1
