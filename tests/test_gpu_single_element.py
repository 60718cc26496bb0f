"""The method's degenerate case: a mesh of one element.  Then P = I and
D = I, so M_bras^-1 = M_br^-1 = M^-1 exactly (eq. mhatinvbras_def): the BRAS
apply must equal a direct solve with the oracle's M, preconditioned CG must
stop after one product M p, and the fixed point with omega = 1 after one
update.  Covered for every element pass of the library (scaled H1 per work-
group and single work-group, per-lane metric form, matrix-core form for
n_loc > 36, FP32 inverses)."""
import sys

import numpy as np
import pytest

from oracle import fe as ofe, assembly as oasm

pytestmark = pytest.mark.gpu

TRI = np.array([[0.1, 0.2], [1.3, 0.1], [0.4, 0.9]])
TET = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 1.1, 0.1], [0.1, 0.3, 1.2]])

CASES = [
    # family, dim, degree, precision
    ("P", 2, 3, "f64"),        # scaled H1, n_loc 10
    ("P", 3, 4, "f64"),        # scaled H1, n_loc 35
    ("N1curl", 3, 2, "f64"),   # metric form per lane, n_loc 20
    ("N1curl", 3, 2, "f32"),   # FP32 inverses
    ("BDM", 2, 3, "f64"),      # n_loc 20
    ("RT", 3, 4, "f64"),       # matrix cores, n_loc 70
]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def ids(c):
    return "%s%d-%dd-%s" % (c[0], c[2], c[1], c[3])


class OneElement:
    """The library's set-up calls on a mesh of one cell (as MassProblem does
    for structured meshes)."""

    def __init__(self, family, dim, degree, prec):
        import torch
        from paper_2607_12138_amd import _lib as L
        self.L = L
        fam = L.FAMILY[family]
        coords = TRI if dim == 2 else TET
        cells = np.arange(dim + 1, dtype=np.int32)[None, :]
        self.n, self.l2g = L.bras_dofmap(fam, dim, degree, len(coords), cells)
        self.n_loc, _ = L.bras_element_info(fam, dim, degree)
        ref = L.bras_reference_mass(fam, dim, degree)
        dev = torch.device("cuda")
        self.coords_d = torch.from_numpy(np.ascontiguousarray(coords)).to(dev)
        self.cells_d = torch.from_numpy(cells).to(dev)
        self.l2g_d = torch.from_numpy(self.l2g).to(dev)
        self.ref_d = torch.from_numpy(np.ascontiguousarray(ref)).to(dev)
        if L.is_h1(fam):
            form, ns = L.ELEM_SCALED_REF, 0
            self.elem_d = torch.empty(1, dtype=torch.float64, device=dev)
        else:
            form, ns = L.ELEM_METRIC_REF, L.nsym(dim)
            self.elem_d = torch.empty((1, ns), dtype=torch.float64, device=dev)
        L.bras_geometry(fam, dim, self.coords_d, self.cells_d, None, self.elem_d)
        self.h = L.bras_setup(self.n, 1, self.n_loc, self.l2g_d, form, self.ref_d, self.elem_d, ns, L.PREC[prec], 1)

    def vec(self):
        import torch
        return torch.zeros(self.n, dtype=torch.float64, device="cuda")

    def close(self):
        self.L.bras_destroy(self.h)


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_single_element_bras_is_the_exact_inverse(case):
    import torch
    family, dim, deg, prec = case
    say("one element %s" % (case,))
    one = OneElement(family, dim, deg, prec)
    L = one.L
    coords = TRI if dim == 2 else TET
    orc = oasm.Problem(ofe.reference_element(family, dim, deg), coords, np.arange(dim + 1)[None, :])
    assert one.n == orc.n == one.n_loc and np.array_equal(one.l2g, orc.pi.astype(np.int32))
    M = orc.M.toarray()
    kappa = np.linalg.cond(M)
    rng = np.random.default_rng(5)
    x = rng.uniform(-1.0, 1.0, one.n)
    y = one.vec()
    L.bras_apply(one.h, torch.from_numpy(x).cuda(), y)
    exact = np.linalg.solve(M, x)
    tol = (10 * kappa * 2.0 ** -53) if prec == "f64" else (10 * kappa * 2.0 ** -24)
    err = np.max(np.abs(y.cpu().numpy() - exact)) / np.max(np.abs(exact))
    assert err <= max(tol, 1e-13), (err, kappa)
    # every multiplicity is 1
    mult = torch.empty(one.n, dtype=torch.int32, device="cuda")
    L.bras_export(one.h, L.EXPORT_MULT, mult)
    assert int(mult.min()) == 1 and int(mult.max()) == 1
    # PCG with BRAS: one product M p (on both solver paths where the small one
    # applies); the first residual is about cond(M) u, u the unit roundoff of
    # the stored inverse (cond(M) <= 250 for these elements)
    rtol = 1e-8 if prec == "f64" else 1e-3
    b = torch.from_numpy(rng.uniform(-1.0, 1.0, one.n)).cuda()
    for small in (1, 0):
        L.bras_set_option(one.h, L.OPT_SMALL_CG, small)
        xs = one.vec()
        st, its, rel = L.pcg_solve(one.h, L.PC_BRAS, b, xs, rtol, 50)
        assert st == L.BRAS_OK and int(its[0]) == 1, (small, its, rel)
        # the fixed point with omega = 1 (C M = I) stops after one update
        xf = one.vec()
        st, its, rel = L.fixed_point_solve(one.h, L.PC_BRAS, 1.0, b, xf, rtol, 50)
        assert st == L.BRAS_OK and int(its[0]) == 1, (small, its, rel)
    one.close()
