"""Assembled operators on the GPU (eq. mass_and_bras_element_sums): the CSR
forms of M and M_bras^-1 built by the library against the oracle's assembled
matrices (pattern bit-exact, values to rounding), and the CSR product against
the oracle and against the matrix-free apply."""
import sys

import numpy as np
import pytest

from oracle import fe as ofe, mesh as omesh, assembly as oasm
import workloads

pytestmark = pytest.mark.gpu

CASES = [
    # family, dim, degree, N, jitter, prec: scaled H1, metric per lane, FP32, packed per element
    ("P", 2, 1, 9, 0.0, "f64"),
    ("P", 3, 3, 3, 0.2, "f64"),
    ("N1curl", 3, 2, 3, 0.2, "f64"),
    ("N1curl", 3, 2, 3, 0.2, "f32"),
    ("RT", 3, 4, 2, 0.2, "f64"),
    ("BDM", 2, 3, 4, 0.2, "f64"),
    ("P", 3, 4, 2, 0.0, "f64"),         # vertex rows: 24 elements x 35 local DOFs
    ("B", 3, 6, 2, 0.2, "f64"),         # degree 6: 24 x 84 = 2016 candidates
]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def ids(c):
    return "%s%d-%dd-N%d-%s" % (c[0], c[2], c[1], c[3], c[5])


def rel_inf(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def to_t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_assembled_operators_match_oracle(case):
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import MassProblem
    family, dim, deg, N, jit, prec = case
    coords, cells = omesh.structured_mesh(dim, N, jitter=jit, seed=11)
    orc = oasm.Problem(ofe.reference_element(family, dim, deg), coords, cells)
    say("setup %s" % (case,))
    gpu = MassProblem(family, dim, deg, N, jitter=jit, seed=11, prec=prec)
    import scipy.sparse as sp
    x = workloads.vector(orc.n, 3)
    # the pattern: every pair of DOFs sharing an element (all-ones element
    # matrices, so no entry cancels)
    pat = oasm.assemble(orc.pi, np.ones_like(orc.mats), orc.n).tocsr()
    pat.sort_indices()
    for op, ref in ((L.OP_MASS, orc.M), (L.OP_BRAS, orc.B)):
        say("assemble op %d" % op)
        rowptr, col, val = gpu.assemble(op)
        rp, cl, vl = rowptr.cpu().numpy(), col.cpu().numpy(), val.cpu().numpy()
        assert np.array_equal(rp, pat.indptr) and np.array_equal(cl, pat.indices)
        ours = sp.csr_matrix((vl, cl, rp), shape=(orc.n, orc.n))
        # BRAS entries come from each side's own float64 inverses: their
        # difference scales with cond(M_K) (large for high-degree Bernstein)
        kappa = np.max(np.linalg.cond(orc.mats)) if op == L.OP_BRAS else 1.0
        tol = 2e-4 if (op == L.OP_BRAS and prec == "f32") else max(1e-14, 10 * kappa * 2.0 ** -53)
        assert abs(ours - ref).max() <= tol * abs(ref).max()
        say("csr apply op %d" % op)
        y = gpu.csr_apply((rowptr, col, val), to_t(x)).cpu().numpy()
        assert rel_inf(y, ref @ x) <= max(tol, 1e-13)
        # the same operator applied matrix-free (whose FP32 form also computes in FP32)
        yf = (gpu.mass if op == L.OP_MASS else gpu.bras)(to_t(x)).cpu().numpy()
        assert rel_inf(y, yf) <= (1e-12 if tol < 1e-13 else tol)


def test_csr_error_paths():
    import torch
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import MassProblem
    gpu = MassProblem("P", 2, 2, 3)
    rowptr, col, val = gpu.assemble(L.OP_MASS)
    with pytest.raises(L.BrasError) as e:
        L.bras_csr_assemble(gpu.h, 7, rowptr, col, val)              # unknown operator
    assert e.value.code == L.BRAS_EINVAL
    x = to_t(workloads.vector(gpu.n, 1))
    with pytest.raises(L.BrasError):
        L.bras_csr_apply(gpu.n, rowptr, col, val, x, x)             # aliasing rejected
    L.bras_csr_apply(0, rowptr, col, val, x, gpu.vec())              # empty: nothing to do
    torch.cuda.synchronize()


def test_bf16_handle_has_no_assembled_bras():
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import MassProblem
    gpu = MassProblem("RT", 3, 2, 2, jitter=0.2, seed=1, prec="bf16")
    with pytest.raises(L.BrasError):
        gpu.assemble(L.OP_BRAS)
