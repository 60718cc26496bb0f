"""Dense spectral checks on tiny problems (pins for the BRAS operator).

kappa_hat(A, B) = lambda_max(B^-1 A) / lambda_min(B^-1 A) (eq. spectral-kappa).
For a preconditioner given by its inverse Binv = B^-1 (SPD) the generalised
eigenvalues of M v = lambda B v are the eigenvalues of L^T M L with
Binv = L L^T (a congruence of Binv M).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def dense(A):
    return A.toarray() if sp.issparse(A) else np.asarray(A, dtype=float)


def preconditioned_eigs(M, Binv):
    """Eigenvalues of Binv M (ascending) for SPD M and SPD Binv."""
    M = dense(M)
    Binv = dense(Binv)
    L = np.linalg.cholesky(Binv)
    return sla.eigvalsh(L.T @ M @ L)


def kappa_hat(M, Binv):
    ev = preconditioned_eigs(M, Binv)
    return ev[-1] / ev[0], ev[0], ev[-1]


def injection(pi, n):
    """P (n_br x n) with P[j, pi(j)] = 1, broken index j = K*n_loc + l."""
    pi = np.asarray(pi).ravel()
    nbr = len(pi)
    return sp.csr_matrix((np.ones(nbr), (np.arange(nbr), pi)), shape=(nbr, n))


def broken_mass(mats):
    return sp.block_diag(list(mats), format="csr")


def copy_constraints(pi, n):
    """C (m x n_br), m = n_br - n, full row rank, ker C = range P: for every
    conforming DOF with broken copies j_1 < ... < j_d, rows w_j1 - w_jt."""
    pi = np.asarray(pi).ravel()
    order = np.argsort(pi, kind="stable")
    rows, cols, vals = [], [], []
    r = 0
    start = 0
    sorted_pi = pi[order]
    while start < len(order):
        stop = start
        while stop < len(order) and sorted_pi[stop] == sorted_pi[start]:
            stop += 1
        first = order[start]
        for t in range(start + 1, stop):
            rows += [r, r]
            cols += [first, order[t]]
            vals += [1.0, -1.0]
            r += 1
        start = stop
    return sp.csr_matrix((vals, (rows, cols)), shape=(r, len(pi)))


def exact_inverse_correction(pi, mats, n):
    """Right-hand side of Lemma bras_exact_inverse_correction:
    M^-1 - Z S^-1 Z^T with S = -C Mbr^-1 C^T, Z = D^-1 P^T Mbr^-1 C^T.
    Returns (that matrix, the correction -Z S^-1 Z^T)."""
    P = dense(injection(pi, n))
    Mbr = dense(broken_mass(mats))
    C = dense(copy_constraints(pi, n))
    Mbr_inv = np.linalg.inv(Mbr)
    D = P.T @ P
    Dinv = np.diag(1.0 / np.diag(D))
    M = P.T @ Mbr @ P
    S = -C @ Mbr_inv @ C.T
    Z = Dinv @ P.T @ Mbr_inv @ C.T
    corr = -Z @ np.linalg.solve(S, Z.T)
    return np.linalg.inv(M) + corr, corr


def projector_lambda_max(pi, mats, n):
    """lambda_max(Mbr Q Mbr^-1 Q), Q = P D^-1 P^T (Thm. bras_lambda_max_projector)."""
    P = dense(injection(pi, n))
    Mbr = dense(broken_mass(mats))
    D = P.T @ P
    Q = P @ np.diag(1.0 / np.diag(D)) @ P.T
    ev = np.linalg.eigvals(Mbr @ Q @ np.linalg.inv(Mbr) @ Q)
    return float(np.max(ev.real))


def metric_contrast(kind, G):
    """beta/alpha bound of Cor. bras_piola_metric_contrast from per-element G."""
    if kind in ("P", "B"):
        return float(np.max(G) / np.min(G))
    ev = np.linalg.eigvalsh(G)
    return float(ev[:, -1].max() / ev[:, 0].min())
