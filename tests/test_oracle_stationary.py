"""Pins for the oracle's fixed-point, Chebyshev and power iterations (Section 3)
against dense eigen-decompositions, the classical contraction bounds the
paper quotes, the Chebyshev polynomial in closed form, and the paper's
printed fixed-point iteration counts."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fe, mesh, assembly, pcg, stationary, spectral
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def problem(family, dim, deg, N, jitter=0.2, seed=3):
    ref = fe.reference_element(family, dim, deg)
    coords, cells = mesh.structured_mesh(dim, N, jitter=jitter, seed=seed)
    return assembly.Problem(ref, coords, cells)


def dense_spectrum(pr, which):
    Cm = np.diag(1.0 / pr.diag) if which == "jacobi" else pr.B.toarray()
    return spectral.preconditioned_eigs(pr.M, Cm), Cm


CASES = [("P", 2, 2, 4), ("RT", 3, 2, 2), ("N1curl", 3, 1, 3)]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("which", ["bras", "jacobi"])
def test_power_iteration_against_eigendecomposition(case, which):
    """With C M v_i = l_i v_i (v_i M-orthogonal, v_i' M v_i = l_i for the
    C^-1-orthonormal generalized eigenvectors) and v0 = sum c_i v_i, the k-th
    estimate is the Rayleigh quotient of (C M)^(k-1) v0:
        sum c_i^2 l_i^(2k) / sum c_i^2 l_i^(2k-1).
    It lies inside the spectrum and does not decrease with k."""
    pr = problem(*case)
    _, Cm = dense_spectrum(pr, which)
    lam, V = sla.eigh(pr.M.toarray(), np.linalg.inv(Cm))
    C = pr.B.dot if which == "bras" else pcg.jacobi(pr.diag)
    v0 = workloads.vector(pr.n, 7)
    c = np.linalg.solve(V, v0)
    s = lam / lam[-1]
    prev = 0.0
    for k in (1, 2, 10, 50, 400):
        est = stationary.power_lambda_max(pr.M, C, v0, iters=k)
        w = c ** 2 * s ** (2 * k - 1)
        closed = lam[-1] * np.sum(w * s) / np.sum(w)
        assert abs(est - closed) <= 1e-9 * lam[-1]
        assert lam[0] * (1 - 1e-12) <= est <= lam[-1] * (1 + 1e-12)
        assert est >= prev * (1 - 1e-12)
        prev = est


@pytest.mark.parametrize("case", CASES)
def test_fixed_point_contracts_at_the_optimal_rate(case):
    """With omega = 2/(lmin + lmax) the energy-norm error shrinks by at least
    (kappa - 1)/(kappa + 1) per update (Section 3's omega_opt)."""
    pr = problem(*case)
    ev, Cm = dense_spectrum(pr, "bras")
    lmin, lmax = ev[0], ev[-1]
    rho = (lmax - lmin) / (lmax + lmin)
    f = workloads.rhs(pr.n, 1, 5)
    Md = pr.M.toarray()
    u_star = np.linalg.solve(Md, f)
    energy = lambda e: np.sqrt(e @ Md @ e)           # noqa: E731
    om = 2.0 / (lmin + lmax)
    prev = energy(u_star)
    for k in range(1, 12):
        u, its, ok, hist = stationary.fixed_point(pr.M, f, pr.B.dot, om, tol=1e-300, maxit=k)
        e = energy(u_star - u)
        assert e <= rho * prev * (1 + 1e-9) + 1e-14 * energy(u_star)
        prev = e


@pytest.mark.parametrize("case", CASES)
def test_chebyshev_matches_polynomial_and_bound(case):
    """e_k = p_k(C M) e_0 with p_k(l) = T_k((theta - l)/delta) / T_k(theta/delta),
    evaluated here through the eigen-decomposition and T_k = cosh(k arccosh .),
    and the bound 2((sqrt(kappa)-1)/(sqrt(kappa)+1))^k the paper quotes."""
    pr = problem(*case)
    ev, Cm = dense_spectrum(pr, "bras")
    lmin, lmax = ev[0], ev[-1]
    Md = pr.M.toarray()
    f = workloads.rhs(pr.n, 1, 6)
    u_star = np.linalg.solve(Md, f)
    # generalized eigenvectors of (M, Cm^-1): C M = V diag(lam) V^-1
    lam, V = sla.eigh(Md, np.linalg.inv(Cm))
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)

    def cheb(k, t):
        t = np.asarray(t, dtype=float)
        out = np.empty_like(t)
        big = np.abs(t) >= 1
        out[big] = np.sign(t[big]) ** k * np.cosh(k * np.arccosh(np.abs(t[big])))
        out[~big] = np.cos(k * np.arccos(t[~big]))
        return out

    kappa = lmax / lmin
    q = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    energy = lambda e: np.sqrt(e @ Md @ e)           # noqa: E731
    c0 = np.linalg.solve(V, u_star)                  # e_0 = u* - 0 in the eigenbasis
    for k in (1, 2, 5, 9):
        u, its, ok, _ = stationary.chebyshev(pr.M, f, pr.B.dot, lmin, lmax, tol=1e-300, maxit=k)
        ek = u_star - u
        pk = cheb(k, (theta - lam) / delta) / cheb(k, np.array([theta / delta]))[0]
        assert np.linalg.norm(ek - V @ (pk * c0)) <= 1e-9 * np.linalg.norm(u_star)
        assert energy(ek) <= 2 * q ** k * energy(u_star) * (1 + 1e-9)


def test_chebyshev_coefficients_closed_form():
    a, b = stationary.chebyshev_coefficients(1.0, 3.0, 6)
    theta, delta = 2.0, 1.0
    sigma = theta / delta
    assert a[0] == 0.0 and b[0] == 1.0 / theta
    # rho_k = T_{k}(sigma) / T_{k+1}(sigma), so a_k = rho_k rho_{k-1}, b_k = 2 rho_k / delta
    T = [1.0, sigma]
    for _ in range(8):
        T.append(2 * sigma * T[-1] - T[-2])
    for k in range(1, 6):
        rk, rkm = T[k] / T[k + 1], T[k - 1] / T[k]
        assert abs(a[k] - rk * rkm) <= 1e-15 and abs(b[k] - 2 * rk / delta) <= 1e-15


def test_iteration_count_definition_and_reduction_to_jacobi_richardson():
    pr = problem("P", 2, 2, 5)
    f = workloads.rhs(pr.n, 1, 2)
    lam = stationary.power_lambda_max(pr.M, pr.B.dot, workloads.vector(pr.n, 7))
    u, its, ok, hist = stationary.fixed_point(pr.M, f, pr.B.dot, 2.0 / (1.0 + lam), tol=1e-10)
    assert ok and len(hist) == its + 1 and hist[-1] <= 1e-10 and all(h > 1e-10 for h in hist[:-1])
    # zero right-hand side: nothing to do
    assert stationary.fixed_point(pr.M, np.zeros(pr.n), pr.B.dot, 0.5)[1] == 0
    # one Chebyshev step equals one fixed-point step with omega = 1/theta
    u1 = stationary.chebyshev(pr.M, f, pr.B.dot, 1.0, lam, tol=1e-300, maxit=1)[0]
    u2 = stationary.fixed_point(pr.M, f, pr.B.dot, 2.0 / (1.0 + lam), tol=1e-300, maxit=1)[0]
    assert np.allclose(u1, u2, rtol=1e-14, atol=0)


@pytest.mark.slow
@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "paper_fixed_point_iterations.json")))["cases"],
                         ids=lambda c: c["cite"])
def test_fixed_point_iterations_match_paper(case):
    pr = problem(case["family"], case["dim"], case["degree"], case["N"], jitter=0.0)
    assert 0.9e6 <= pr.n <= 1.1e6
    f = workloads.rhs(pr.n, 1, 1)
    v0 = workloads.vector(pr.n, 7)
    Cd = pcg.jacobi(pr.diag)
    lam_d = stationary.power_lambda_max(pr.M, Cd, v0)
    lam_b = stationary.power_lambda_max(pr.M, pr.B.dot, v0)
    _, it_d, ok_d, _ = stationary.fixed_point(pr.M, f, Cd, 1.0 / lam_d, tol=1e-10)
    _, it_b, ok_b, _ = stationary.fixed_point(pr.M, f, pr.B.dot, 2.0 / (1.0 + lam_b), tol=1e-10)
    assert ok_d and ok_b
    assert abs(it_d - case["its_diag"]) <= 3 and abs(it_b - case["its_bras"]) <= 3
