"""Damped fixed-point iteration, Chebyshev iteration and the power iteration
that sets their parameters (Section 3, mass-solve numerics).

Test infrastructure: a plain NumPy statement of what the library's stationary
solvers compute.

Fixed point (Section 3):  u_{k+1} = u_k + omega C (f - M u_k), C in
{diag(M)^-1, M_bras^-1}.  Weights used in the paper:
    omega_diag = 1 / lambda_max(C M),
    omega_bras = 2 / (1 + lambda_max(C M))   (lambda_min >= 1, Cor. bras_lambda_min).
lambda_max is estimated with the power iteration.  Both solvers start from
u_0 (zero in the paper) and stop when ||f - M u_k||_2 <= tol ||f - M u_0||_2,
returning k, the number of updates, or after maxit updates.

Readings where the paper is silent (listed in the design notes):
* power iteration: v_0 = v0 / ||v0||; for k = 1..iters: w = C M v_{k-1},
  lambda_k = (M v_{k-1}) . w / (M v_{k-1}) . v_{k-1}  (Rayleigh quotient of
  the M-self-adjoint operator C M), v_k = w / ||w||; the estimate is
  lambda_iters.  The start vector is a seeded U[-1,1] vector, iters = 50.
* Chebyshev iteration (the paper recommends it for its CG-like rate without
  dot products; it does not fix a form): the three-term Chebyshev
  semi-iteration for C M on [lmin, lmax] (e.g. Saad, Iterative Methods for
  Sparse Linear Systems, 2nd ed., Alg. 12.1), applied to the true residual:
      theta = (lmax + lmin)/2, delta = (lmax - lmin)/2, sigma = theta/delta
      d_0 = C r_0 / theta,  rho_0 = 1/sigma
      u_{k+1} = u_k + d_k
      rho_{k+1} = 1 / (2 sigma - rho_k)
      d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1} / delta) C r_{k+1}
  with r_k = f - M u_k.  For BRAS, lmin = 1 (Cor. bras_lambda_min).
"""
import numpy as np


def _mv(A):
    return A.dot if hasattr(A, "dot") else A


def power_lambda_max(M, apply_C, v0, iters=50):
    """Power-iteration estimate of lambda_max(C M) (reading above)."""
    matvec = _mv(M)
    v = np.asarray(v0, dtype=float)
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        q = matvec(v)
        w = apply_C(q)
        lam = (q @ w) / (q @ v)
        v = w / np.linalg.norm(w)
    return lam


def chebyshev_coefficients(lmin, lmax, count):
    """(a_k, b_k), k < count, of the update d_k = a_k d_{k-1} + b_k C r_k."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    a = np.zeros(count)
    b = np.zeros(count)
    if count == 0:
        return a, b
    b[0] = 1.0 / theta
    rho = 1.0 / sigma
    for k in range(1, count):
        rho_new = 1.0 / (2.0 * sigma - rho)
        a[k] = rho_new * rho
        b[k] = 2.0 * rho_new / delta
        rho = rho_new
    return a, b


def fixed_point(M, f, apply_C, omega, x0=None, tol=1e-10, maxit=5000):
    """Damped fixed point; returns (u, updates, converged, history of ||r_k||/||r_0||)."""
    matvec = _mv(M)
    f = np.asarray(f, dtype=float)
    u = np.zeros_like(f) if x0 is None else np.array(x0, dtype=float)
    r = f - matvec(u)
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return u, 0, True, hist
    for k in range(maxit + 1):
        rel = np.linalg.norm(r) / r0
        if k > 0:
            hist.append(rel)
        if rel <= tol:
            return u, k, True, hist
        if k == maxit:
            break
        u = u + omega * apply_C(r)
        r = f - matvec(u)
    return u, maxit, False, hist


def chebyshev(M, f, apply_C, lmin, lmax, x0=None, tol=1e-10, maxit=5000):
    """Chebyshev semi-iteration on [lmin, lmax]; same return values as fixed_point."""
    matvec = _mv(M)
    f = np.asarray(f, dtype=float)
    u = np.zeros_like(f) if x0 is None else np.array(x0, dtype=float)
    r = f - matvec(u)
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return u, 0, True, hist
    a, b = chebyshev_coefficients(lmin, lmax, maxit)
    d = np.zeros_like(f)
    for k in range(maxit + 1):
        rel = np.linalg.norm(r) / r0
        if k > 0:
            hist.append(rel)
        if rel <= tol:
            return u, k, True, hist
        if k == maxit:
            break
        d = a[k] * d + b[k] * apply_C(r)
        u = u + d
        r = f - matvec(u)
    return u, maxit, False, hist
