"""Element matrices, conforming mass matrix, Jacobi and the BRAS operator.

Element mass matrices follow the Piola pullbacks (eq. piola_mass_pullbacks):
  H1      M_K = rho_K |det J_K| Mhat
  H(curl) M_K = sum_ab G_ab Mhat^{ab},  G = rho_K |det J_K| J_K^-1 J_K^-T
  H(div)  M_K = sum_ab G_ab Mhat^{ab},  G = rho_K J_K^T J_K / |det J_K|
(|det J| because cells list vertices in ascending order, which need not be
orientation preserving; the sign cancels in every mass integrand).

Conforming mass (eq. M_PMbrP): M = P^T M_br P = sum_K P_K^T M_K P_K.
Diagonal preconditioner (Section 2.1): M_diag^-1 = diag(M)^-1.
BRAS (eqs. mhatinvbras_def, mass_and_bras_element_sums):
  M_bras^-1 = D^-1 (sum_K P_K^T M_K^-1 P_K) D^-1,  D = P^T P.
"""
import numpy as np
import scipy.sparse as sp

from .mesh import jacobians


def metric(kind, coords, cells, rho=None):
    """Per-element pullback coefficient G_K: [E] for H1, [E, d, d] otherwise."""
    J = jacobians(coords, cells)
    det = np.linalg.det(J)
    adet = np.abs(det)
    r = np.ones(len(cells)) if rho is None else np.asarray(rho, dtype=float)
    if kind == "P":
        return r * adet
    if kind == "N1curl":
        Jinv = np.linalg.inv(J)
        return (r * adet)[:, None, None] * (Jinv @ np.transpose(Jinv, (0, 2, 1)))
    if kind == "RT":
        return (r / adet)[:, None, None] * (np.transpose(J, (0, 2, 1)) @ J)
    raise ValueError(kind)


def element_matrices(ref, coords, cells, rho=None):
    """M_K for every element, [E, n_loc, n_loc]."""
    G = metric(ref.family, coords, cells, rho)
    if ref.family == "P":
        return G[:, None, None] * ref.mass[None]
    return np.einsum("kab,abij->kij", G, ref.mass)


def assemble(pi, mats, n):
    """sum_K P_K^T A_K P_K as CSR (A_K = mats[K])."""
    E, nl = pi.shape
    rows = np.repeat(pi, nl, axis=1).ravel()
    cols = np.tile(pi, (1, nl)).ravel()
    A = sp.coo_matrix((mats.reshape(E, -1).ravel(), (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def element_inverses(mats):
    """Exact local inverses M_K^-1 via Cholesky (fails loudly if M_K is not SPD)."""
    L = np.linalg.cholesky(mats)
    Linv = np.linalg.inv(L)
    return np.transpose(Linv, (0, 2, 1)) @ Linv


def mass_matrix(pi, mats, n):
    return assemble(pi, mats, n)


def bras_matrix(pi, mats, n, d=None):
    """Explicitly assembled M_bras^-1 = D^-1 (sum_K P_K^T M_K^-1 P_K) D^-1 (CSR)."""
    if d is None:
        d = np.bincount(pi.ravel(), minlength=n)
    S = assemble(pi, element_inverses(mats), n)
    Dinv = sp.diags(1.0 / d)
    return (Dinv @ S @ Dinv).tocsr()


def bras_apply_matrix_free(pi, inv_mats, d, x):
    """y = D^-1 P^T M_br^-1 P D^-1 x without assembling (second route, for cross-checks)."""
    x = np.asarray(x, dtype=float)
    n = len(d)
    s = x / d if x.ndim == 1 else x / d[:, None]
    w = s[pi]                                                    # [E, n_loc(, R)]
    if x.ndim == 1:
        z = np.einsum("kij,kj->ki", inv_mats, w)
        y = np.bincount(pi.ravel(), weights=z.ravel(), minlength=n)
        return y / d
    z = np.einsum("kij,kjr->kir", inv_mats, w)
    y = np.zeros((n, x.shape[1]))
    np.add.at(y, pi.ravel(), z.reshape(-1, x.shape[1]))
    return y / d[:, None]


def mass_apply_matrix_free(pi, mats, x):
    """y = P^T M_br P x element by element (second route, for cross-checks)."""
    n = len(x)
    w = np.asarray(x, dtype=float)[pi]
    z = np.einsum("kij,kj->ki", mats, w)
    return np.bincount(pi.ravel(), weights=z.ravel(), minlength=n)


class Problem:
    """Everything the oracle derives for one (mesh, element) pair."""

    def __init__(self, ref, coords, cells, rho=None, need_bras=True):
        from .dofmap import build_dofmap, multiplicity
        self.ref = ref
        self.coords = coords
        self.cells = cells
        self.pi, self.n, self.offsets = build_dofmap(cells, len(coords), ref.dofs_per_entity)
        self.d = multiplicity(self.pi, self.n)
        self.mats = element_matrices(ref, coords, cells, rho)
        self.M = mass_matrix(self.pi, self.mats, self.n)
        self.diag = self.M.diagonal().copy()
        self.B = bras_matrix(self.pi, self.mats, self.n, self.d) if need_bras else None

    @property
    def n_br(self):
        return self.pi.size
