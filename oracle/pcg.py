"""Textbook preconditioned conjugate gradients (Section 3).

The paper solves M u = f from u_0 = 0 and stops when the residual
r_k = f - M u_k satisfies ||r_k||_2 / ||r_0||_2 <= tol, or after 5000
iterations.  The iteration count returned is the number of products M p
performed when the test first passes (reading: the recursive residual is the
one tested inside the loop).

    x = x0; r = b - M x; z = C r; p = z; rho = r.z
    for k = 1..maxit:
        q = M p; alpha = rho / p.q; x += alpha p; r -= alpha q
        if ||r|| / ||r0|| <= tol: stop with k
        z = C r; rho' = r.z; p = z + (rho'/rho) p; rho = rho'

`flexible=True` replaces beta by r_new.(z_new - z_old) / rho_old
(Polak-Ribiere form), the usual safeguard when C is applied inexactly.
"""
import numpy as np


def pcg(M, b, apply_C=None, x0=None, tol=1e-10, maxit=5000, flexible=False):
    """Return (x, iterations, converged, history of ||r_k||/||r_0||)."""
    b = np.asarray(b, dtype=float)
    matvec = M.dot if hasattr(M, "dot") else M
    C = (lambda v: v) if apply_C is None else apply_C
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=float)
    r = b - matvec(x)
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return x, 0, True, hist
    z = C(r)
    p = z.copy()
    rho = r @ z
    for k in range(1, maxit + 1):
        q = matvec(p)
        alpha = rho / (p @ q)
        x += alpha * p
        r -= alpha * q
        rel = np.linalg.norm(r) / r0
        hist.append(rel)
        if rel <= tol:
            return x, k, True, hist
        z_new = C(r)
        rho_new = r @ z_new
        if flexible:
            beta = (r @ (z_new - z)) / rho
        else:
            beta = rho_new / rho
        p = z_new + beta * p
        z = z_new
        rho = rho_new
    return x, maxit, False, hist


def jacobi(diag):
    d = np.asarray(diag, dtype=float)
    return lambda v: v / d


def cg_iteration_bound(kappa, tol):
    """Smallest k with 2((sqrt(kappa)-1)/(sqrt(kappa)+1))^k <= tol (Section 3, CG
    rate estimate); the paper notes observed CG rates follow this closely."""
    s = np.sqrt(kappa)
    rate = (s - 1.0) / (s + 1.0)
    if rate <= 0.0:
        return 1
    return int(np.ceil(np.log(tol / 2.0) / np.log(rate)))
