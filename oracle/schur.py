"""Schur-complement approximations built from an approximate mass inverse
(Section 4, block preconditioning).

Test infrastructure: a plain SciPy statement of what the library's sparse
products compute.

For the symmetric saddle-point matrix [[M, G^T], [G, -C]] (eq.
saddle_matrix_general_22, C symmetric positive semi-definite) the positive
Schur complement is -S = C + G M^-1 G^T (eq. positive_schur_general), and
replacing M^-1 by a sparse SPD approximation Mt^-1 (M_bras^-1, or diag(M)^-1)
gives -St = C + G Mt^-1 G^T (eq. approx_positive_schur_general), sparse
when Mt^-1 is.  The constants of eq. schur_a0-c0 are the extreme generalised
eigenvalues of (G Mt^-1 G^T, G M^-1 G^T).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def schur_approx(G, Minv, C=None):
    """-St = C + G Minv G^T (sparse products; Minv sparse or dense)."""
    G = sp.csr_matrix(G)
    S = G @ (Minv @ G.T)
    S = sp.csr_matrix(S) if not sp.issparse(S) else S.tocsr()
    if C is not None:
        S = S + sp.csr_matrix(C)
    return S


def exact_schur(G, M, C=None):
    """-S = C + G M^-1 G^T, dense (small problems)."""
    Gd = G.toarray() if sp.issparse(G) else np.asarray(G, dtype=float)
    Md = M.toarray() if sp.issparse(M) else np.asarray(M, dtype=float)
    S = Gd @ np.linalg.solve(Md, Gd.T)
    if C is not None:
        S = S + (C.toarray() if sp.issparse(C) else np.asarray(C, dtype=float))
    return 0.5 * (S + S.T)


def generalized_extremes(A, B):
    """(lambda_min, lambda_max) of A v = lambda B v for symmetric A and SPD B."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=float)
    B = B.toarray() if sp.issparse(B) else np.asarray(B, dtype=float)
    ev = sla.eigh(0.5 * (A + A.T), 0.5 * (B + B.T), eigvals_only=True)
    return ev[0], ev[-1]


def alpha0_beta0(G, M, Minv):
    """alpha_0, beta_0 of eq. schur_a0-c0 (G of full row rank): the extreme
    generalised eigenvalues of (G Minv G^T, G M^-1 G^T)."""
    return generalized_extremes(schur_approx(G, Minv), exact_schur(G, M))
