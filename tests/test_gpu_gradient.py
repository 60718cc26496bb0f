"""GPU parity of the differentiable mass solve x = M(rho)^-1 b (H1 P4, density
per element, M_K = rho_K |det J_K| Mhat, eq. h1_mass_pullback): the
per-element contraction, the autograd wrapper against the oracle's adjoint
gradient, finite differences by difference solves, the closed-form
identities, and the full-size 32^3 P4 system with lognormal densities.

Tolerances: the GPU gradient against the oracle's (direct solves) within
1e-8 of max |dL/drho| at CG tolerance 1e-12 (the oracle's own PCG at 1e-12
is within about 1e-12 on the 6^3 mesh, so this leaves room for the rounding
order of the device); finite differences within 1e-6 of |dL/drho_K| on each of
64 sampled elements (central differences with h = 1e-4 rho_K are accurate to
about h^2 relative); the identities within 1e-10.
"""
import sys
import time

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fe as ofe, mesh as omesh, assembly as oasm, gradient as ograd
import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


_CACHE = {}


def setup(deg=4, N=6, seed=21):
    key = (deg, N, seed)
    if key in _CACHE:
        return _CACHE[key]
    from paper_2607_12138_amd.problem import MassProblem
    coords, cells = omesh.structured_mesh(3, N)
    E = len(cells)
    rho = workloads.density(E, seed)
    ref = ofe.reference_element("P", 3, deg)
    orc = oasm.Problem(ref, coords, cells, rho=rho)
    unit = oasm.element_matrices(ref, coords, cells)
    say("gradient setup P%d N=%d (n=%d)" % (deg, N, orc.n))
    gpu = MassProblem("P", 3, deg, N, rho=rho)
    b = workloads.rhs(orc.n, 1, seed + 1)
    xs = workloads.target(orc.n, seed + 2)
    lu = spla.splu(orc.M.tocsc())
    _CACHE[key] = (orc, unit, gpu, rho, b, xs, lu)
    return _CACHE[key]


def t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def refined_solver(lu):
    """Solves A y = rhs for A close to the factored M (a rank-n_loc change of
    relative size 1e-4): LU of M as the preconditioner of a few refinement
    steps, to rounding level."""
    def solve(A, rhs):
        y = lu.solve(rhs)
        for _ in range(8):
            dy = lu.solve(rhs - A @ y)
            y += dy
            if np.linalg.norm(dy) <= 1e-15 * np.linalg.norm(y):
                break
        return y
    return solve


def oracle_gradient(orc, unit, lu, b, xs):
    x = lu.solve(b)
    lam = lu.solve(x - xs)
    return x, lam, ograd.rho_gradient(orc.pi, unit, x, lam)


def test_rho_grad_contraction():
    orc, unit, gpu, rho, b, xs, lu = setup()
    x = workloads.vector(orc.n, 5)
    lam = workloads.vector(orc.n, 6)
    say("bras_rho_grad")
    g = gpu.rho_grad(t(x), t(lam)).cpu().numpy()
    want = ograd.rho_gradient(orc.pi, unit, x, lam)
    assert np.max(np.abs(g - want)) <= 1e-12 * np.max(np.abs(want))


def test_autograd_gradient_against_oracle_fd_and_identities():
    import torch
    from paper_2607_12138_amd.autograd import mass_solve
    orc, unit, gpu, rho, b, xs, lu = setup()
    gpu.set_density(t(rho))
    say("autograd forward/backward (P4 6^3, rtol 1e-12)")
    bt = t(b).requires_grad_(True)
    rt = t(rho).requires_grad_(True)
    x = mass_solve(bt, rt, gpu, 1e-12)
    loss = 0.5 * torch.sum((x - t(xs)) ** 2)
    loss.backward()
    gb = bt.grad.cpu().numpy()
    gr = rt.grad.cpu().numpy()
    xo, lam, gro = oracle_gradient(orc, unit, lu, b, xs)
    eb = np.max(np.abs(gb - lam)) / np.max(np.abs(lam))
    er = np.max(np.abs(gr - gro)) / np.max(np.abs(gro))
    say("  dL/db rel. error %.2e, dL/drho rel. error %.2e" % (eb, er))
    assert eb <= 1e-8
    assert er <= 1e-8
    xg = x.detach().cpu().numpy()
    gvec = xg - xs
    # homogeneity of M(rho): sum_K rho_K dL/drho_K = -(x - x*)^T x ; symmetry: lambda^T b = (x - x*)^T x
    assert abs(rho @ gr + gvec @ xg) <= 1e-10 * abs(gvec @ xg)
    assert abs(gb @ b - gvec @ xg) <= 1e-10 * abs(gvec @ xg)
    # central finite differences (oracle difference solves) on 64 sampled elements
    solve = refined_solver(lu)
    worst = 0.0
    for K in workloads.sample(len(rho), 64, 9):
        fd = ograd.fd_rho(solve, orc.M, orc.pi, unit, xo, xs, K, 1e-4 * rho[K])
        rel = abs(fd - gr[K]) / abs(gr[K])
        worst = max(worst, rel)
        assert rel <= 1e-6, (K, fd, gr[K])
    say("  finite differences: worst rel. error %.2e on 64 elements" % worst)


def test_backward_uses_the_density_of_its_forward():
    """Two forward solves with different densities, then backward through the
    first: the adjoint runs with the first density (the problem object held
    the second one in between)."""
    import torch
    from paper_2607_12138_amd.autograd import mass_solve
    orc, unit, gpu, rho, b, xs, lu = setup()
    rho2 = workloads.density(len(rho), 1234)
    say("two forwards, backward through the first")
    rt = t(rho).requires_grad_(True)
    x1 = mass_solve(t(b), rt, gpu, 1e-12)
    x2 = mass_solve(t(b), t(rho2), gpu, 1e-12)
    loss = 0.5 * torch.sum((x1 - t(xs)) ** 2)
    loss.backward()
    _, _, gro = oracle_gradient(orc, unit, lu, b, xs)
    er = np.max(np.abs(rt.grad.cpu().numpy() - gro)) / np.max(np.abs(gro))
    assert er <= 1e-8, er
    del x2


def test_set_density_updates_operator():
    orc, unit, gpu, rho, b, xs, lu = setup(deg=2, N=3)
    rho2 = workloads.density(len(rho), 99)
    say("set_density")
    gpu.set_density(t(rho2))
    orc2 = oasm.Problem(ofe.reference_element("P", 3, 2), orc.coords, orc.cells, rho=rho2)
    x = workloads.vector(orc.n, 4)
    ym = gpu.mass(t(x)).cpu().numpy()
    yb = gpu.bras(t(x)).cpu().numpy()
    assert np.max(np.abs(ym - orc2.M @ x)) <= 1e-13 * np.max(np.abs(orc2.M @ x))
    assert np.max(np.abs(yb - orc2.B @ x)) <= 1e-13 * np.max(np.abs(orc2.B @ x))


def test_fullsize_gradient_central_differences():
    """The 32^3 x 6 P4 system with rho ~ lognormal(0, 1) (2.1M DOFs): dL/drho
    from autograd (BRAS-PCG at rtol 1e-12, forward and adjoint) against
    central differences on 64 sampled elements, each from two difference
    solves M(rho +- h e_K) dx = -+ h P_K^T M_K^(1) P_K x on the device
    (Jacobi-PCG at rtol 1e-12, an independent solver), with M_K^(1) = |det J_K|
    Mhat from the oracle's element matrices: L(rho +- h e_K) - L(rho) =
    (x - x*)^T dx + ||dx||^2 / 2.  The error of g^T dx from the difference
    solve is lambda^T r for its final residual r, at most about 1e-12 |lambda|
    |rhs|, far below the 1e-6 tolerance."""
    import torch
    from paper_2607_12138_amd.problem import MassProblem
    from paper_2607_12138_amd.autograd import mass_solve
    w = workloads.BY_NAME["h1p4_3d_32_rho"]
    rho = workloads.density(w.n_cells, w.seed(2))
    say("full-size gradient: setup 32^3 P4")
    gpu = MassProblem("P", 3, 4, w.N, jitter=w.jitter, seed=w.mesh_seed, rho=rho)
    n = gpu.n
    b = t(workloads.rhs(n, 1, w.seed(1)))
    xs = t(workloads.target(n, w.seed(3)))
    bt = b.clone().requires_grad_(True)
    rt = t(rho).requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = mass_solve(bt, rt, gpu, 1e-12)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss = 0.5 * torch.sum((x - xs) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    say("  forward %.1f ms, backward %.1f ms" % ((t1 - t0) * 1e3, (t2 - t1) * 1e3))
    gr = rt.grad.cpu().numpy()
    xh = x.detach().cpu().numpy()
    g = xh - xs.cpu().numpy()
    # oracle element matrices of the sampled elements (mesh rebuilt on the oracle side)
    coords, cells = omesh.structured_mesh(3, w.N, jitter=w.jitter, seed=w.mesh_seed)
    assert np.array_equal(cells, gpu.cells)
    ref = ofe.reference_element("P", 3, 4)
    Ks = workloads.sample(len(rho), 64, w.seed(4))
    unit = oasm.element_matrices(ref, coords, cells[Ks])
    say("  central differences on 64 elements")
    worst = 0.0
    for j, K in enumerate(Ks):
        h = 1e-4 * rho[K]
        idx = gpu.l2g[K]
        ax = unit[j] @ xh[idx]
        dL = []
        for sgn in (1.0, -1.0):
            r2 = rho.copy()
            r2[K] += sgn * h
            gpu.set_density(t(r2))
            rhs = np.zeros(n)
            rhs[idx] = -sgn * h * ax
            dx, st, its, rel = gpu.solve(t(rhs), "jacobi", rtol=1e-12)
            assert st == 0
            dx = dx.cpu().numpy()
            dL.append(g @ dx + 0.5 * dx @ dx)
        fd = (dL[0] - dL[1]) / (2.0 * h)
        err = abs(fd - gr[K]) / abs(gr[K])
        worst = max(worst, err)
        assert err <= 1e-6, (K, fd, gr[K])
    say("  finite differences: worst rel. error %.2e on 64 elements" % worst)
    gpu.close()
