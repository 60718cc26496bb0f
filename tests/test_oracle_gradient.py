"""Pins for the oracle's density gradient: finite differences and closed-form identities."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import fe, mesh, assembly, gradient
import workloads


def setup(N=2, deg=3, seed=5):
    ref = fe.reference_element("P", 3, deg)
    coords, cells = mesh.structured_mesh(3, N)
    rho = workloads.density(len(cells), seed)
    pr = assembly.Problem(ref, coords, cells, rho=rho)
    unit = assembly.element_matrices(ref, coords, cells)          # M_K^(1) = |det J| Mhat
    b = workloads.rhs(pr.n, 1, seed + 1)
    xstar = workloads.target(pr.n, seed + 2)
    return pr, unit, rho, b, xstar


def solve(A, r):
    return spla.spsolve(A.tocsc(), r)


def test_gradient_against_central_differences():
    pr, unit, rho, b, xstar = setup()
    x = solve(pr.M, b)
    lam = solve(pr.M, x - xstar)
    g = gradient.rho_gradient(pr.pi, unit, x, lam)
    for K in workloads.sample(len(rho), 12, 77):
        fd = gradient.fd_rho(solve, pr.M, pr.pi, unit, x, xstar, K, 1e-4 * rho[K])
        assert abs(fd - g[K]) <= 1e-6 * max(abs(g[K]), 1e-3 * np.abs(g).max())


def test_gradient_identities():
    pr, unit, rho, b, xstar = setup()
    x = solve(pr.M, b)
    gvec = x - xstar
    lam = solve(pr.M, gvec)
    g = gradient.rho_gradient(pr.pi, unit, x, lam)
    # M(rho) is homogeneous of degree one in rho: sum_K rho_K dL/drho_K = -(x - x*)^T x
    assert abs(rho @ g + gvec @ x) <= 1e-10 * abs(gvec @ x)
    # symmetry of M: lambda^T b = (x - x*)^T x
    assert abs(lam @ b - gvec @ x) <= 1e-10 * abs(gvec @ x)


def test_rhs_gradient_is_exact_for_quadratic_loss():
    pr, unit, rho, b, xstar = setup(N=2, deg=2)
    x = solve(pr.M, b)
    lam = solve(pr.M, x - xstar)
    v = workloads.vector(pr.n, 9)
    eps = 1e-3

    def loss(bb):
        xx = solve(pr.M, bb)
        return 0.5 * np.sum((xx - xstar) ** 2)
    fd = (loss(b + eps * v) - loss(b - eps * v)) / (2 * eps)
    assert abs(fd - lam @ v) <= 1e-7 * abs(lam @ v)
