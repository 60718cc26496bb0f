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
    if kind in ("P", "B"):          # H1 (Lagrange or Bernstein basis)
        return r * adet
    if kind in ("N1curl", "N2curl"):          # covariant Piola
        Jinv = np.linalg.inv(J)
        return (r * adet)[:, None, None] * (Jinv @ np.transpose(Jinv, (0, 2, 1)))
    if kind in ("RT", "BDM"):                 # contravariant Piola
        return (r / adet)[:, None, None] * (np.transpose(J, (0, 2, 1)) @ J)
    raise ValueError(kind)


def element_matrices(ref, coords, cells, rho=None):
    """M_K for every element, [E, n_loc, n_loc]."""
    G = metric(ref.family, coords, cells, rho)
    if ref.family in ("P", "B"):
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


def operator_rows(ref, coords, cells, pi, n, rows, x, which, rho=None):
    """Selected rows of M x ("mass") or M_bras^-1 x ("bras") computed one by one
    from the element-sum definitions (eqs. M_PMbrP, mass_and_bras_element_sums):
        (M x)_i        = sum_{(K,l): pi(K,l) = i} (M_K x[pi_K])_l
        (Mbras^-1 x)_i = d_i^-1 sum_{(K,l): pi(K,l) = i} (M_K^-1 (x/d)[pi_K])_l
    Only the elements touching the requested rows are formed (for sampled
    checks at full size).  x is [n] or [n, R]."""
    from .mesh import jacobians
    pi = np.asarray(pi)
    rows = np.asarray(rows)
    d = np.bincount(pi.ravel(), minlength=n).astype(float)
    x = np.asarray(x, dtype=float)
    xs = x / (d if x.ndim == 1 else d[:, None]) if which == "bras" else x
    flat = pi.ravel()
    order = np.argsort(flat, kind="stable")
    starts = np.searchsorted(flat[order], rows, side="left")
    stops = np.searchsorted(flat[order], rows, side="right")
    out = np.zeros((len(rows),) + x.shape[1:])
    for t, (a, b) in enumerate(zip(starts, stops)):
        for j in order[a:b]:
            K, l = divmod(int(j), pi.shape[1])
            sub_rho = None if rho is None else np.asarray(rho)[K:K + 1]
            MK = element_matrices(ref, coords, cells[K:K + 1], sub_rho)[0]
            if which == "bras":
                MK = element_inverses(MK[None])[0]
            out[t] += MK[l] @ xs[pi[K]]
        if which == "bras":
            out[t] /= d[rows[t]]
    return out
