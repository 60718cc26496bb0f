"""A conforming mass system on a structured simplicial mesh, built and solved
entirely by libbras (mesh, numbering and reference tables on the host side of
the library; geometry, maps, element inverses, operators and PCG in HIP
kernels).  torch provides device memory and the stream only.
"""
import numpy as np

from . import _lib as L


class MassProblem:
    def __init__(self, family, dim, degree, N, jitter=0.0, seed=0, rho=None, prec="f64", max_rhs=1,
                 device="cuda", coord_map=None):
        import torch
        self.family = L.FAMILY[family] if isinstance(family, str) else family
        self.dim, self.degree, self.N = dim, degree, N
        self.prec = L.PREC[prec] if isinstance(prec, str) else prec
        self.max_rhs = max_rhs
        self.device = torch.device(device)
        self.coords, self.cells = L.bras_mesh_structured(dim, N, jitter, seed)
        if coord_map is not None:          # e.g. an affine map of the whole mesh
            self.coords = np.ascontiguousarray(coord_map(self.coords), dtype=np.float64)
        self.n, self.l2g = L.bras_dofmap(self.family, dim, degree, len(self.coords), self.cells)
        self.n_loc, self.dofs_per_entity = L.bras_element_info(self.family, dim, degree)
        self.E = len(self.cells)
        self.ref = L.bras_reference_mass(self.family, dim, degree)
        dev = self.device
        self.coords_d = torch.from_numpy(self.coords).to(dev)
        self.cells_d = torch.from_numpy(self.cells).to(dev)
        self.l2g_d = torch.from_numpy(self.l2g).to(dev)
        self.ref_d = torch.from_numpy(np.ascontiguousarray(self.ref)).to(dev)
        if L.is_h1(self.family):
            self.form, self.nsym = L.ELEM_SCALED_REF, 0
            self.elem_d = torch.empty(self.E, dtype=torch.float64, device=dev)
            self.dcoef_d = torch.empty(self.E, dtype=torch.float64, device=dev)
            L.bras_geometry(self.family, dim, self.coords_d, self.cells_d, None, self.dcoef_d)
        else:
            self.form, self.nsym = L.ELEM_METRIC_REF, L.nsym(dim)
            self.elem_d = torch.empty((self.E, self.nsym), dtype=torch.float64, device=dev)
            self.dcoef_d = None
        self.rho_d = None if rho is None else torch.as_tensor(np.asarray(rho, dtype=np.float64), device=dev)
        L.bras_geometry(self.family, dim, self.coords_d, self.cells_d, self.rho_d, self.elem_d)
        self.h = L.bras_setup(self.n, self.E, self.n_loc, self.l2g_d, self.form, self.ref_d, self.elem_d, self.nsym,
                              self.prec, max_rhs)

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) is not None:
            L.bras_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- operators ---------------------------------------------------------
    def vec(self, nrhs=1):
        import torch
        shape = (self.n,) if nrhs == 1 else (self.n, nrhs)
        return torch.zeros(shape, dtype=torch.float64, device=self.device)

    def bras(self, x, y=None):
        y = self.vec(1 if x.dim() == 1 else x.shape[1]) if y is None else y
        L.bras_apply(self.h, x, y)
        return y

    def mass(self, x, y=None):
        y = self.vec(1 if x.dim() == 1 else x.shape[1]) if y is None else y
        L.mass_apply(self.h, x, y)
        return y

    def jacobi(self, x, y=None):
        y = self.vec(1 if x.dim() == 1 else x.shape[1]) if y is None else y
        L.jacobi_apply(self.h, x, y)
        return y

    def solve(self, b, pc="bras", rtol=1e-10, maxit=5000, x0=None):
        """Returns (x, status, iterations, true relative residuals)."""
        pcode = {"none": L.PC_NONE, "jacobi": L.PC_JACOBI, "bras": L.PC_BRAS}[pc]
        x = self.vec(1 if b.dim() == 1 else b.shape[1]) if x0 is None else x0.clone()
        st, its, rel = L.pcg_solve(self.h, pcode, b, x, rtol, maxit)
        return x, st, its, rel

    # -- stationary iterations (Section 3) ------------------------------------
    def lambda_max(self, pc="bras", v0=None, iters=50):
        """Power-iteration estimate of lambda_max(C M)."""
        import torch
        if v0 is None:
            raise ValueError("a start vector is required (seeded, e.g. workloads.vector)")
        v0 = torch.as_tensor(v0, dtype=torch.float64, device=self.device)
        return L.bras_lambda_max(self.h, L.PC[pc], v0, iters)

    def fixed_point(self, b, pc="bras", omega=None, rtol=1e-10, maxit=5000, x0=None):
        """Damped fixed point; returns (x, status, updates, relres)."""
        x = self.vec(1 if b.dim() == 1 else b.shape[1]) if x0 is None else x0.clone()
        st, its, rel = L.fixed_point_solve(self.h, L.PC[pc], omega, b, x, rtol, maxit)
        return x, st, its, rel

    def chebyshev(self, b, pc="bras", lmin=1.0, lmax=None, rtol=1e-10, maxit=5000, x0=None):
        """Chebyshev semi-iteration on [lmin, lmax]; returns (x, status, updates, relres)."""
        x = self.vec(1 if b.dim() == 1 else b.shape[1]) if x0 is None else x0.clone()
        st, its, rel = L.chebyshev_solve(self.h, L.PC[pc], lmin, lmax, b, x, rtol, maxit)
        return x, st, its, rel

    def set_density(self, rho_d):
        """Recompute element coefficients rho_K |det J_K| and the inverses (H1)."""
        self.rho_d = rho_d
        L.bras_geometry(self.family, self.dim, self.coords_d, self.cells_d, rho_d, self.elem_d)
        L.bras_update(self.h, self.elem_d)

    def rho_grad(self, x, lam, g=None):
        import torch
        g = torch.empty(self.E, dtype=torch.float64, device=self.device) if g is None else g
        L.bras_rho_grad(self.h, x, lam, self.dcoef_d, g)
        return g

    def info(self, what):
        return L.bras_info(self.h, what)

    def autotune(self, nrhs=None):
        """Pick the fastest element-pass scheduling variant for this mesh."""
        L.bras_autotune(self.h, self.max_rhs if nrhs is None else nrhs)
        return L.bras_info(self.h, "variant")

    def assemble(self, op):
        """The assembled operator (L.OP_MASS, L.OP_BRAS or L.OP_JACOBI) as CSR
        device tensors (rowptr int64, col int32, val float64)."""
        import torch
        rowptr = torch.empty(self.n + 1, dtype=torch.int64, device=self.device)
        if op == L.OP_JACOBI:
            col = torch.empty(self.n, dtype=torch.int32, device=self.device)
            val = torch.empty(self.n, dtype=torch.float64, device=self.device)
            L.bras_csr_jacobi(self.h, rowptr, col, val)
            return rowptr, col, val
        nnz = L.bras_csr_rowptr(self.h, rowptr)
        col = torch.empty(nnz, dtype=torch.int32, device=self.device)
        val = torch.empty(nnz, dtype=torch.float64, device=self.device)
        L.bras_csr_assemble(self.h, op, rowptr, col, val)
        return rowptr, col, val

    def csr_apply(self, csr, x, y=None):
        y = self.vec() if y is None else y
        L.bras_csr_apply(self.n, csr[0], csr[1], csr[2], x, y)
        return y

    def export(self, what):
        import torch
        if what == L.EXPORT_MULT:
            out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        elif what == L.EXPORT_ROWPTR:
            out = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        elif what == L.EXPORT_SLOT:
            out = torch.empty(self.E * self.n_loc, dtype=torch.int64, device=self.device)
        else:
            out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        L.bras_export(self.h, what, out)
        return out

    def schur(self, G, op=None, C=None):
        """-St = C + G Mt^-1 G^T (Section 4, eq. approx_positive_schur_general)
        for a CSR coupling G = (rowptr, col, val) of shape m x n on the device,
        Mt^-1 the assembled operator op (default L.OP_BRAS) and an optional
        CSR C (m x m): the sparse products (G Mt^-1) G^T, then the sum with C.
        Returns the CSR of -St (m x m)."""
        op = L.OP_BRAS if op is None else op
        m = G[0].numel() - 1
        Bop = self.assemble(op)
        T = spgemm(G, Bop, m, self.n)
        Gt = csr_transpose(G, m, self.n)
        S = spgemm(T, Gt, m, self.n)
        return S if C is None else csr_add(S, C, m)


def spgemm(a, b, m, k):
    """C = A B for CSR device tensors a (m x k) and b (k x n), each
    (rowptr int64, col int32, val float64); returns C as such a triple."""
    import torch
    dev = a[0].device
    if a[1].numel() == 0 or b[1].numel() == 0:
        return (torch.zeros(m + 1, dtype=torch.int64, device=dev), torch.empty(0, dtype=torch.int32, device=dev),
                torch.empty(0, dtype=torch.float64, device=dev))
    rp = torch.empty(m + 1, dtype=torch.int64, device=dev)
    nnz = L.bras_spgemm_rowptr(m, k, a, b, rp)
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
    L.bras_spgemm_fill(m, k, a, b, (rp, col, val))
    return rp, col[:nnz], val[:nnz]


def csr_transpose(a, m, n):
    """A^T (n x m) of a CSR device triple a (m x n)."""
    import torch
    dev = a[0].device
    nnz = a[1].numel()
    rp = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
    if nnz == 0:
        return torch.zeros(n + 1, dtype=torch.int64, device=dev), col[:0], val[:0]
    L.bras_csr_transpose(m, n, a, (rp, col, val))
    return rp, col, val


def csr_add(a, b, m):
    """A + B for CSR device triples of the same shape (m rows)."""
    import torch
    dev = a[0].device
    if a[1].numel() == 0:
        return b
    if b[1].numel() == 0:
        return a
    rp = torch.empty(m + 1, dtype=torch.int64, device=dev)
    nnz = L.bras_csr_add_rowptr(m, a, b, rp)
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
    L.bras_csr_add_fill(m, a, b, (rp, col, val))
    return rp, col[:nnz], val[:nnz]
