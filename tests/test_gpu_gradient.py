"""GPU parity of the differentiable mass solve x = M(rho)^-1 b (H1, density per
element): the per-element contraction, the autograd wrapper against the
oracle's adjoint gradient, finite differences and closed-form identities."""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fe as ofe, mesh as omesh, assembly as oasm, gradient as ograd
import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def setup(deg=4, N=3, seed=21):
    import torch
    from paper_2607_12138_amd.problem import MassProblem
    coords, cells = omesh.structured_mesh(3, N)
    E = len(cells)
    rho = workloads.density(E, seed)
    ref = ofe.reference_element("P", 3, deg)
    orc = oasm.Problem(ref, coords, cells, rho=rho)
    unit = oasm.element_matrices(ref, coords, cells)
    say("gradient setup P%d N=%d" % (deg, N))
    gpu = MassProblem("P", 3, deg, N, rho=rho)
    b = workloads.rhs(orc.n, 1, seed + 1)
    xs = workloads.target(orc.n, seed + 2)
    return orc, unit, gpu, rho, b, xs


def t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_rho_grad_contraction():
    orc, unit, gpu, rho, b, xs = setup()
    x = workloads.vector(orc.n, 5)
    lam = workloads.vector(orc.n, 6)
    say("bras_rho_grad")
    g = gpu.rho_grad(t(x), t(lam)).cpu().numpy()
    want = ograd.rho_gradient(orc.pi, unit, x, lam)
    assert np.max(np.abs(g - want)) <= 1e-12 * np.max(np.abs(want))


def test_autograd_gradient_against_oracle_and_identities():
    import torch
    from paper_2607_12138_amd.autograd import mass_solve
    orc, unit, gpu, rho, b, xs = setup()
    say("autograd forward/backward")
    bt = t(b).requires_grad_(True)
    rt = t(rho).requires_grad_(True)
    x = mass_solve(bt, rt, gpu, 1e-12)
    loss = 0.5 * torch.sum((x - t(xs)) ** 2)
    loss.backward()
    gb = bt.grad.cpu().numpy()
    gr = rt.grad.cpu().numpy()
    solve = lambda A, r: spla.spsolve(A.tocsc(), r)
    xo = solve(orc.M, b)
    lam = solve(orc.M, xo - xs)
    gro = ograd.rho_gradient(orc.pi, unit, xo, lam)
    assert np.max(np.abs(gb - lam)) <= 1e-7 * np.max(np.abs(lam))
    assert np.max(np.abs(gr - gro)) <= 1e-7 * np.max(np.abs(gro))
    xg = x.detach().cpu().numpy()
    gvec = xg - xs
    # homogeneity of M(rho): sum_K rho_K dL/drho_K = -(x - x*)^T x ; symmetry: lambda^T b = (x - x*)^T x
    assert abs(rho @ gr + gvec @ xg) <= 1e-9 * abs(gvec @ xg)
    assert abs(gb @ b - gvec @ xg) <= 1e-9 * abs(gvec @ xg)
    # central finite differences (oracle difference solves) on a few elements
    for K in workloads.sample(len(rho), 6, 9):
        fd = ograd.fd_rho(solve, orc.M, orc.pi, unit, xo, xs, K, 1e-4 * rho[K])
        assert abs(fd - gr[K]) <= 1e-6 * max(abs(gr[K]), 1e-3 * np.max(np.abs(gr)))


def test_set_density_updates_operator():
    orc, unit, gpu, rho, b, xs = setup(deg=2, N=3)
    rho2 = workloads.density(len(rho), 99)
    say("set_density")
    gpu.set_density(t(rho2))
    orc2 = oasm.Problem(ofe.reference_element("P", 3, 2), orc.coords, orc.cells, rho=rho2)
    x = workloads.vector(orc.n, 4)
    ym = gpu.mass(t(x)).cpu().numpy()
    yb = gpu.bras(t(x)).cpu().numpy()
    assert np.max(np.abs(ym - orc2.M @ x)) <= 1e-13 * np.max(np.abs(orc2.M @ x))
    assert np.max(np.abs(yb - orc2.B @ x)) <= 1e-13 * np.max(np.abs(orc2.B @ x))
