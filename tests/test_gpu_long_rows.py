"""A conforming DOF with more broken copies than one reduce chunk holds (2048):
a synthetic map of 3000 elements that all contain DOF 0, each with three DOFs
of its own, and seeded SPD element matrices (explicit form).  DOF 0 then has
d_0 = 3000 copies, and its row of the transpose map is summed straight from
device memory instead of through the chunk's LDS buffer.  The BRAS apply
D^-1 P^T M_br^-1 P D^-1 (eq. mhatinvbras_def), the mass apply P^T M_br P
(eq. M_PMbrP) and the preconditioned CG (whose fused epilogues take the same
branch) are checked against the oracle's assembled operators."""
import sys

import numpy as np
import pytest

from oracle import assembly as oasm, pcg as opcg
import workloads

pytestmark = pytest.mark.gpu

E, NL = 3000, 4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def star_system(seed=17):
    n = 1 + 3 * E
    pi = np.empty((E, NL), dtype=np.int64)
    pi[:, 0] = 0
    pi[:, 1:] = 1 + 3 * np.arange(E)[:, None] + np.arange(3)[None, :]
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1.0, 1.0, size=(E, NL, NL))
    mats = A @ A.transpose(0, 2, 1) + NL * np.eye(NL)[None]
    return n, pi, mats


def oracle_ops(n, pi, mats):
    d = np.bincount(pi.ravel(), minlength=n).astype(float)
    M = oasm.assemble(pi, mats, n)
    inv = oasm.element_inverses(mats)
    Dinv = 1.0 / d
    B = oasm.assemble(pi, inv, n).multiply(Dinv[:, None]).multiply(Dinv[None, :]).tocsr()
    return M, B, d


@pytest.fixture(scope="module")
def system():
    import torch
    from paper_2607_12138_amd import _lib as L
    n, pi, mats = star_system()
    M, B, d = oracle_ops(n, pi, mats)
    assert d[0] == E > 2048
    dev = torch.device("cuda")
    l2g_d = torch.from_numpy(pi.astype(np.int32)).to(dev)
    elem_d = torch.from_numpy(np.ascontiguousarray(mats)).to(dev)
    say("long-row system: n=%d E=%d, d_0=%d" % (n, E, int(d[0])))
    h = L.bras_setup(n, E, NL, l2g_d, L.ELEM_EXPLICIT, None, elem_d, 0, L.FP64, 3)
    yield L, h, n, M, B
    L.bras_destroy(h)


@pytest.mark.parametrize("R", [1, 3])
def test_long_row_applies(system, R):
    import torch
    L, h, n, M, B = system
    X = workloads.rhs(n, R, 40 + R)
    x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    shape = (n,) if R == 1 else (n, R)
    say("long-row bras_apply / mass_apply R=%d" % R)
    for fn, op in ((L.bras_apply, B), (L.mass_apply, M)):
        y = torch.zeros(shape, dtype=torch.float64, device="cuda")
        fn(h, x, y)
        want = op @ X
        got = y.cpu().numpy()
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)), fn.__name__
        # the long row itself (a sum of 3000 copies)
        assert np.all(np.abs(got[0] - want[0]) <= 1e-13 * np.max(np.abs(want))), fn.__name__


def test_long_row_pcg(system):
    import torch
    L, h, n, M, B = system
    b = workloads.rhs(n, 1, 47)
    say("long-row BRAS-PCG")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    st, its, rel = L.pcg_solve(h, L.PC_BRAS, torch.from_numpy(b).cuda(), x, 1e-10, 500)
    assert st == L.BRAS_OK
    xo, ito, ok, _ = opcg.pcg(M, b, B.dot, tol=1e-10)
    assert ok and abs(int(its[0]) - ito) <= 1, (its, ito)
    xg = x.cpu().numpy()
    assert np.linalg.norm(b - M @ xg) <= 1e-10 * np.linalg.norm(b)
