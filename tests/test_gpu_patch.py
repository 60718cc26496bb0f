"""The patch form of the one-column operator passes (gather, element products
and LDS sums per patch of elements, shared DOFs summed by a second pass):
BRAS (eq. mhatinvbras_def) and mass (eq. M_PMbrP) applies against the oracle's
assembled operators, against the element / reduce passes of the same handle,
bit-for-bit repeatable, and inside CG (where the vectors use the plan's
internal DOF numbering) against the oracle's iteration counts.  Cases: every
per-lane form (packed float32 / float64 inverses, 2D and 3D metric tables,
explicit element matrices), the scaled H1 form on the matrix cores (patch form
on request), small patches (many shared DOFs, several ranks per patch), one
element per patch, and a single patch without shared DOFs (no boundary pass)."""
import os
import sys

import numpy as np
import pytest

from oracle import fe as ofe, mesh as omesh, assembly as oasm, pcg as opcg
import workloads

pytestmark = pytest.mark.gpu

CASES = [
    # family, dim, degree, N, jitter, prec, environment
    ("N1curl", 3, 2, 5, 0.2, "f32", {}),
    ("N1curl", 3, 2, 4, 0.2, "f64", {}),
    ("RT", 3, 3, 3, 0.2, "f64", {}),
    ("BDM", 2, 2, 7, 0.2, "f64", {}),
    ("N1curl", 2, 4, 6, 0.2, "f32", {}),
    ("N1curl", 3, 2, 4, 0.2, "f64", {"BRAS_PATCH_ELEMS": "7"}),
    ("RT", 3, 2, 4, 0.2, "f32", {"BRAS_PATCH_ELEMS": "33", "BRAS_PATCH_XCD": "0"}),
    ("P", 3, 3, 4, 0.2, "f64", {"BRAS_PATCH_SCALED": "1"}),
    ("P", 3, 4, 3, 0.0, "f64", {"BRAS_PATCH_SCALED": "1", "BRAS_PATCH_ELEMS": "64"}),
    ("P", 2, 2, 9, 0.2, "f64", {"BRAS_PATCH_SCALED": "1", "BRAS_PATCH_ELEMS": "5"}),
    ("N1curl", 3, 2, 2, 0.2, "f64", {}),                               # one patch, no shared DOFs
    ("RT", 3, 2, 3, 0.2, "f32", {"BRAS_PATCH_ELEMS": "1"}),             # one element per patch
    ("P", 3, 2, 2, 0.0, "f64", {"BRAS_PATCH_SCALED": "1"}),            # scaled form, one patch
]


def ids(c):
    return "%s%d-%dd-N%d-%s%s" % (c[0], c[2], c[1], c[3], c[5], "".join("-%s%s" % (k[11:].lower(), v)
                                                                         for k, v in c[6].items()))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_inf(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def build(case):
    from paper_2607_12138_amd.problem import MassProblem
    family, dim, deg, N, jit, prec, env = case
    seed = 2000 + N
    coords, cells = omesh.structured_mesh(dim, N, jitter=jit, seed=seed)
    orc = oasm.Problem(ofe.reference_element(family, dim, deg), coords, cells)
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        gpu = MassProblem(family, dim, deg, N, jitter=jit, seed=seed, prec=prec)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return orc, gpu


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_patch_operators(case):
    from paper_2607_12138_amd import _lib as L
    say("patch form %s" % (case,))
    orc, gpu = build(case)
    assert gpu.info("patches") > 0
    if case[6].get("BRAS_PATCH_ELEMS") == "1":
        assert gpu.info("patches") == gpu.E
    if case[3] == 2:
        assert gpu.info("patches") == 1
    tb = 1e-13 if case[5] == "f64" else 2e-4
    x = workloads.vector(orc.n, 41)
    xd = to_t(x)
    yb = gpu.bras(xd).cpu().numpy()
    ym = gpu.mass(xd).cpu().numpy()
    assert rel_inf(ym, orc.M @ x) <= 1e-13
    assert rel_inf(yb, orc.B @ x) <= tb
    # repeatable bit for bit
    assert np.array_equal(yb.view(np.uint64), gpu.bras(xd).cpu().numpy().view(np.uint64))
    # the element / reduce passes of the same handle agree to rounding
    L.bras_set_option(gpu.h, L.OPT_PATCH, 0)
    yb0 = gpu.bras(xd).cpu().numpy()
    ym0 = gpu.mass(xd).cpu().numpy()
    L.bras_set_option(gpu.h, L.OPT_PATCH, 1)
    assert rel_inf(ym, ym0) <= 1e-13
    assert rel_inf(yb, yb0) <= (1e-13 if case[5] == "f64" else 1e-6)
    # CG in the internal numbering, both preconditioners, against the oracle
    b = workloads.rhs(orc.n, 1, 42)
    rtol = 1e-10 if case[5] == "f64" else 1e-8
    for pc, C in (("bras", orc.B.dot), ("jacobi", lambda v: v / orc.diag)):
        xg, st, its, rel = gpu.solve(to_t(b), pc, rtol=rtol)
        assert st == L.BRAS_OK, (pc, L.bras_last_error())
        xo, ito, ok, _ = opcg.pcg(orc.M, b, C, tol=rtol)
        xg = xg.cpu().numpy()
        assert np.linalg.norm(b - orc.M @ xg) <= rtol * np.linalg.norm(b)
        if case[5] == "f64":
            assert abs(int(its[0]) - ito) <= 1, (pc, its, ito)
        say("  %s: %d iterations (oracle %d)" % (pc, int(its[0]), ito))
    gpu.close()


def test_patch_stationary_and_lambda():
    """The fixed point and the Chebyshev iteration (their residual and update
    passes in patch form) and the power iteration on a patch-form handle."""
    from paper_2607_12138_amd import _lib as L
    from oracle import stationary as ost
    orc, gpu = build(("N1curl", 3, 2, 4, 0.2, "f64", {}))
    v0 = workloads.vector(orc.n, 43)
    lam_g = gpu.lambda_max("bras", v0, 50)
    lam_o = ost.power_lambda_max(orc.M, orc.B.dot, v0, 50)
    assert abs(lam_g - lam_o) <= 1e-10 * lam_o
    b = workloads.rhs(orc.n, 1, 44)
    xg, st, its, rel = gpu.fixed_point(to_t(b), "bras", 2.0 / (1.0 + lam_g), rtol=1e-8)
    assert st == L.BRAS_OK and rel[0] <= 1e-8
    xo, ito, ok = ost.fixed_point(orc.M, b, orc.B.dot, 2.0 / (1.0 + lam_o), tol=1e-8)[:3]
    assert abs(int(its[0]) - ito) <= 1
    xg, st, its, rel = gpu.chebyshev(to_t(b), "bras", 1.0, 1.02 * lam_g, rtol=1e-8)
    assert st == L.BRAS_OK and rel[0] <= 1e-8
    gpu.close()
