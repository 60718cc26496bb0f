"""Gradient of a density-dependent mass solve (oracle side).

x(rho, b) = M(rho)^-1 b with M(rho) = sum_K rho_K P_K^T M_K^(1) P_K and
M_K^(1) = |det J_K| Mhat (H1, eq. h1_mass_pullback), loss
L = 0.5 ||x - x*||^2.  With g = x - x* and the adjoint lambda = M^-1 g
(M is symmetric):
    dL/db      = lambda
    dL/drho_K  = -lambda_K^T M_K^(1) x_K.

Finite differences use difference solves to avoid cancellation:
    M(rho +- h e_K) dx = -+ h P_K^T M_K^(1) P_K x,
    L(rho +- h e_K) - L(rho) = g^T dx + 0.5 ||dx||^2.
"""
import numpy as np
import scipy.sparse as sp


def rho_gradient(pi, mats_unit, x, lam):
    """dL/drho_K = -lambda_K^T M_K^(1) x_K for every K (mats_unit = M_K^(1))."""
    return -np.einsum("ki,kij,kj->k", lam[pi], mats_unit, x[pi])


def element_operator(pi, mats_unit, K, n):
    """P_K^T M_K^(1) P_K as a sparse n x n matrix."""
    idx = pi[K]
    nl = len(idx)
    rows = np.repeat(idx, nl)
    cols = np.tile(idx, nl)
    return sp.csr_matrix((mats_unit[K].ravel(), (rows, cols)), shape=(n, n))


def fd_rho(solve, M, pi, mats_unit, x, xstar, K, h):
    """Central difference of L in rho_K by difference solves.

    solve(A, rhs) must return A^-1 rhs to high accuracy.
    """
    n = len(x)
    g = x - xstar
    A1 = element_operator(pi, mats_unit, K, n)
    rhs = A1 @ x
    out = []
    for sgn in (+1.0, -1.0):
        Ms = M + sgn * h * A1
        dx = solve(Ms, -sgn * h * rhs)
        out.append(g @ dx + 0.5 * dx @ dx)
    return (out[0] - out[1]) / (2.0 * h)
