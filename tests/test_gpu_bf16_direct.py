"""Plain BF16 Gram-factor applies with the single-copy epilogue (DOFs with
one broken copy, e.g. cell-interior and boundary-face DOFs, are written to y
by the element pass and skipped by the reduce) against the same handle type
without it: BRAS applies (eq. mhatinvbras_def) bit for bit at 1, 32 and 40
columns (40: more than one 32-column block, where the epilogue is off), and
solves, power iteration and fixed point (which keep the broken vector for
every DOF) unchanged bit for bit."""
import os
import sys

import numpy as np
import pytest

from oracle import fe as ofe, mesh as omesh, assembly as oasm
import workloads

pytestmark = pytest.mark.gpu

CASES = [("RT", 3, 4, 2, 0.2), ("RT", 3, 2, 3, 0.2), ("N1curl", 3, 2, 3, 0.0)]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make(case, direct):
    from paper_2607_12138_amd.problem import MassProblem
    family, dim, deg, N, jit = case
    old = os.environ.get("BRAS_BF16_DIRECT")
    os.environ["BRAS_BF16_DIRECT"] = "1" if direct else "0"
    try:
        return MassProblem(family, dim, deg, N, jitter=jit, seed=3000 + N, prec="bf16", max_rhs=40)
    finally:
        if old is None:
            os.environ.pop("BRAS_BF16_DIRECT", None)
        else:
            os.environ["BRAS_BF16_DIRECT"] = old


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s%d-%dd-N%d" % (c[0], c[2], c[1], c[3]))
def test_bf16_single_copy_epilogue(case):
    from paper_2607_12138_amd import _lib as L
    family, dim, deg, N, jit = case
    say("bf16 single-copy epilogue %s" % (case,))
    on, off = make(case, True), make(case, False)
    coords, cells = omesh.structured_mesh(dim, N, jitter=jit, seed=3000 + N)
    orc = oasm.Problem(ofe.reference_element(family, dim, deg), coords, cells)
    assert orc.n == on.n
    single = int(np.sum(np.asarray(orc.d) == 1))   # DOFs with one broken copy
    assert single > 0   # the case exercises the epilogue
    for R in (1, 32, 40):
        X = to_t(workloads.rhs(on.n, R, 70 + R))
        a = on.bras(X).cpu().numpy()
        b = off.bras(X).cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), R
    # the solvers' passes do not take the epilogue: identical results
    Bm = to_t(workloads.rhs(on.n, 32, 71))
    Xa, sa, ia, ra = on.solve(Bm, "bras", rtol=1e-8)
    Xb, sb, ib, rb = off.solve(Bm, "bras", rtol=1e-8)
    assert sa == L.BRAS_OK and sb == L.BRAS_OK
    assert np.array_equal(np.asarray(ia), np.asarray(ib))
    assert np.array_equal(Xa.cpu().numpy().view(np.uint64), Xb.cpu().numpy().view(np.uint64))
    Xa = Xa.cpu().numpy()
    Bh = Bm.cpu().numpy()
    for r in range(0, 32, 5):
        true_rel = np.linalg.norm(Bh[:, r] - orc.M @ Xa[:, r]) / np.linalg.norm(Bh[:, r])
        assert true_rel <= 1.5e-8
    v0 = workloads.vector(on.n, 73)
    lam, lam0 = on.lambda_max("bras", v0, 30), off.lambda_max("bras", v0, 30)
    assert lam == lam0
    b1 = to_t(workloads.rhs(on.n, 1, 72))
    xs1, ss1, is1, rs1 = on.fixed_point(b1, "bras", 2.0 / (1.0 + lam), rtol=1e-6, maxit=3000)
    xs0, ss0, is0, rs0 = off.fixed_point(b1, "bras", 2.0 / (1.0 + lam), rtol=1e-6, maxit=3000)
    assert ss1 == L.BRAS_OK and ss0 == L.BRAS_OK and int(is1[0]) == int(is0[0])
    assert np.array_equal(xs1.cpu().numpy().view(np.uint64), xs0.cpu().numpy().view(np.uint64))
    on.close()
    off.close()


def test_local_gemm_microbenchmark_runs():
    """The LDS-resident microbenchmark of the BF16 Gram products: runs for every
    covered n_loc, reports the issued FLOPs of the launch, and its per-thread
    checksums are finite and repeatable (the products are deterministic)."""
    import torch
    from paper_2607_12138_amd import _lib as L
    for nl in (20, 36, 70, 84):
        out = torch.empty(8 * 256, dtype=torch.float32, device="cuda")
        fl = L.bras_bench_bf16_local_gemm(nl, 3, 8, out)
        assert fl == 3 * 8 * L.bras_bench_bf16_local_gemm(nl, 1, 0)
        a = out.cpu().numpy().copy()
        L.bras_bench_bf16_local_gemm(nl, 3, 8, out)
        b = out.cpu().numpy()
        assert np.all(np.isfinite(a)) and np.array_equal(a, b)
