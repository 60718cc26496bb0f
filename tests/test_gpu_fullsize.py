"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times: sampled rows of the mass and BRAS operators against the
oracle's row-by-row element sums, and PCG to the workload tolerance."""
import sys

import numpy as np
import pytest

from oracle import fe as ofe, mesh as omesh, assembly as oasm, dofmap as odofmap, pcg as opcg
import workloads

pytestmark = pytest.mark.gpu

FULL = [w for w in workloads.WORKLOADS if w.prec != "bf16"]
BF16 = [w for w in workloads.WORKLOADS if w.prec == "bf16"]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("w", FULL, ids=lambda w: w.name)
def test_sampled_rows_and_solve(w):
    import torch
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import MassProblem
    ref = ofe.reference_element(w.family, w.dim, w.degree)
    coords, cells = omesh.structured_mesh(w.dim, w.N, jitter=w.jitter, seed=w.mesh_seed)
    rho = workloads.density(len(cells), w.seed(2)) if w.density else None
    pi, n, _ = odofmap.build_dofmap(cells, len(coords), ref.dofs_per_entity)
    say("full-size setup %s n=%d E=%d" % (w.name, n, len(cells)))
    gpu = MassProblem(w.family, w.dim, w.degree, w.N, jitter=w.jitter, seed=w.mesh_seed, rho=rho, prec=w.prec)
    assert gpu.n == n and np.array_equal(gpu.l2g, pi.astype(np.int32))
    variant = gpu.autotune(w.nrhs)        # the element-pass variant the benchmark times with
    say("  autotuned variant %d" % variant)
    x = workloads.vector(n, w.seed(4))
    rows = workloads.sample(n, 48, w.seed(4))
    say("  sampled mass/bras rows")
    ym = gpu.mass(torch.from_numpy(x).cuda()).cpu().numpy()
    yb = gpu.bras(torch.from_numpy(x).cuda()).cpu().numpy()
    om = oasm.operator_rows(ref, coords, cells, pi, n, rows, x, "mass", rho=rho)
    ob = oasm.operator_rows(ref, coords, cells, pi, n, rows, x, "bras", rho=rho)
    assert np.max(np.abs(ym[rows] - om)) <= 1e-13 * np.max(np.abs(ym))
    tol_b = 1e-13 if w.prec == "f64" else 2e-4
    assert np.max(np.abs(yb[rows] - ob)) <= tol_b * np.max(np.abs(yb))
    b = workloads.rhs(n, w.nrhs, w.seed(1))
    say("  pcg bras / jacobi")
    bt = torch.from_numpy(b).cuda()
    for pc in ("bras", "jacobi"):
        xs, st, its, rel = gpu.solve(bt, pc, rtol=w.tol)
        assert st == L.BRAS_OK
        r = bt - gpu.mass(xs)
        true_rel = float(torch.linalg.norm(r) / torch.linalg.norm(bt))
        assert true_rel <= w.tol * 1.5 and abs(true_rel - rel[0]) <= 1e-3 * w.tol
        say("  %s: %d iterations, true relres %.3e" % (pc, its[0], true_rel))
    gpu.close()


@pytest.mark.parametrize("name", ["h1p1_2d_32", "h1p3_3d_24_jit"])
def test_iteration_counts_match_oracle_at_full_size(name):
    import torch
    from paper_2607_12138_amd.problem import MassProblem
    w = workloads.BY_NAME[name]
    ref = ofe.reference_element(w.family, w.dim, w.degree)
    coords, cells = omesh.structured_mesh(w.dim, w.N, jitter=w.jitter, seed=w.mesh_seed)
    orc = oasm.Problem(ref, coords, cells)
    b = workloads.rhs(orc.n, 1, w.seed(1))
    say("full-size oracle pcg %s" % name)
    gpu = MassProblem(w.family, w.dim, w.degree, w.N, jitter=w.jitter, seed=w.mesh_seed)
    for pc, C in (("bras", orc.B.dot), ("jacobi", opcg.jacobi(orc.diag))):
        xo, ito, ok, _ = opcg.pcg(orc.M, b, C, tol=w.tol)
        x, st, its, rel = gpu.solve(torch.from_numpy(b).cuda(), pc, rtol=w.tol)
        assert abs(int(its[0]) - ito) <= 1
        xg = x.cpu().numpy()
        assert np.linalg.norm(xg - xo) <= 1e-8 * np.linalg.norm(xo)
    gpu.close()


def _bf16_rows(ref, coords, cells, pi, n, rows, X):
    """Rows of the emulated BF16 Gram-factor apply, from the elements touching them."""
    from oracle import reduced
    flat = pi.ravel()
    touch = np.unique(np.nonzero(np.isin(flat, rows))[0] // pi.shape[1])
    mats = oasm.element_matrices(ref, coords, cells[touch])
    d = np.bincount(flat, minlength=n)
    G = reduced.round_bf16(reduced.gram_factors(mats, pi[touch], d))
    w = reduced.round_bf16(X[pi[touch]])
    U = reduced.round_bf16(np.einsum("kij,kjr->kir", G, w))
    Z = np.einsum("kji,kjr->kir", G, U)
    out = np.zeros((len(rows), X.shape[1]))
    where = {int(r): t for t, r in enumerate(rows)}
    for e, K in enumerate(touch):
        for l, i in enumerate(pi[K]):
            if int(i) in where:
                out[where[int(i)]] += Z[e, l]
    return out


@pytest.mark.parametrize("w", BF16, ids=lambda w: w.name)
def test_bf16_multi_rhs_full_size(w):
    import torch
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import MassProblem
    ref = ofe.reference_element(w.family, w.dim, w.degree)
    coords, cells = omesh.structured_mesh(w.dim, w.N, jitter=w.jitter, seed=w.mesh_seed)
    pi, n, _ = odofmap.build_dofmap(cells, len(coords), ref.dofs_per_entity)
    say("full-size setup %s n=%d E=%d R=%d" % (w.name, n, len(cells), w.nrhs))
    gpu = MassProblem(w.family, w.dim, w.degree, w.N, jitter=w.jitter, seed=w.mesh_seed, prec=w.prec,
                      max_rhs=w.nrhs)
    assert gpu.n == n
    X = workloads.rhs(n, w.nrhs, w.seed(4))
    rows = workloads.sample(n, 24, w.seed(4))
    Xt = torch.from_numpy(X).cuda()
    say("  sampled rows (bf16 emulation, float64 mass)")
    Yb = gpu.bras(Xt).cpu().numpy()
    Ym = gpu.mass(Xt).cpu().numpy()
    eb = _bf16_rows(ref, coords, cells, pi, n, rows, X)
    diff = np.abs(Yb[rows] - eb)
    assert np.mean(diff > 1e-5 * np.max(np.abs(Yb))) < 0.02
    assert np.max(diff) <= 1e-2 * np.max(np.abs(Yb))
    om = oasm.operator_rows(ref, coords, cells, pi, n, rows, X, "mass")
    assert np.max(np.abs(Ym[rows] - om)) <= 1e-13 * np.max(np.abs(Ym))
    del Yb, Ym
    b = workloads.rhs(n, w.nrhs, w.seed(1))
    bt = torch.from_numpy(b).cuda()
    say("  flexible pcg, %d columns" % w.nrhs)
    xs, st, its, rel = gpu.solve(bt, "bras", rtol=w.tol)
    assert st == L.BRAS_OK
    r = bt - gpu.mass(xs)
    true_rel = (torch.linalg.norm(r, dim=0) / torch.linalg.norm(bt, dim=0)).cpu().numpy()
    assert np.all(true_rel <= w.tol * 1.5)
    say("  iterations %s restarts %d" % (list(its), gpu.info("restarts")))
    gpu.close()
