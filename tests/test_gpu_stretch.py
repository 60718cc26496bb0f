"""GPU side of the rotated-stretch study (eq. rot_stretch_map): operator parity
with the oracle on stretched meshes and high-degree 2D BDM (n_loc 42 and 72 on
the matrix cores), the power-iteration lambda_max against the oracle's, and
the metric-contrast bound of Cor. bras_piola_metric_contrast on the GPU's own
estimates."""
import sys

import numpy as np
import pytest

from oracle import fe as ofe, mesh as omesh, assembly as oasm, stationary as ost
import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_inf(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def to_t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pair(deg, N, r, prec="f64"):
    from paper_2607_12138_amd.problem import MassProblem
    coords, cells = omesh.structured_mesh(2, N, jitter=0.0, seed=0)
    orc = oasm.Problem(ofe.reference_element("BDM", 2, deg), workloads.rotated_stretch(coords, r), cells)
    say("setup BDM%d N=%d r=%g %s" % (deg, N, r, prec))
    gpu = MassProblem("BDM", 2, deg, N, prec=prec, coord_map=lambda x: workloads.rotated_stretch(x, r))
    assert np.array_equal(gpu.coords, orc.coords)
    return orc, gpu


@pytest.mark.parametrize("deg,N,r,prec", [(3, 5, 3.0, "f64"), (1, 9, 7.0, "f64"), (5, 3, 5.0, "f64"),
                                          (7, 3, 3.0, "f64"), (7, 3, 1.0, "f32")])
def test_stretched_operators_match(deg, N, r, prec):
    orc, gpu = pair(deg, N, r, prec)
    x = workloads.vector(orc.n, 17)
    say("mass / bras apply")
    # a stretched, high-degree M x cancels heavily: bound the error by the
    # product of absolute values (the usual float64 dot-product bound)
    ym = gpu.mass(to_t(x)).cpu().numpy()
    assert np.max(np.abs(ym - orc.M @ x)) <= 1e-13 * np.max(abs(orc.M) @ np.abs(x))
    err = rel_inf(gpu.bras(to_t(x)).cpu().numpy(), orc.B @ x)
    # both sides invert M_K in their own float64 order: the difference scales
    # with cond(M_K), which the stretch multiplies by up to r^4
    kappa = np.max(np.linalg.cond(orc.mats))
    tol = max(1e-13, 10 * kappa * 2.0 ** -53) if prec == "f64" else max(2e-4, 10 * kappa * 2.0 ** -24)
    assert err <= tol, (err, kappa)


@pytest.mark.parametrize("pc", ["bras", "jacobi"])
def test_stretched_lambda_max_matches_oracle(pc):
    from oracle import pcg as opcg
    orc, gpu = pair(3, 5, 3.0)
    v0 = workloads.vector(orc.n, 5)
    C = orc.B.dot if pc == "bras" else opcg.jacobi(orc.diag)
    lo = ost.power_lambda_max(orc.M, C, v0, iters=50)
    say("lambda_max %s" % pc)
    lg = gpu.lambda_max(pc, v0, 50)
    assert abs(lg - lo) <= 1e-10 * lo


def test_metric_contrast_bound_on_gpu_estimates():
    """lambda_max(r) <= r^4 lambda_max(1) for BRAS (its lambda_min is 1), with
    the GPU's power-iteration estimates at about 5e3 DOFs."""
    from paper_2607_12138_amd import stretch
    base = stretch.run_case(3, 1.0)
    say(str(base))
    for r in (3.0, 5.0):
        st = stretch.run_case(3, r)
        say(str(st))
        assert base["lambda_max"][1] < st["lambda_max"][1] <= r ** 4 * base["lambda_max"][1] * 1.001
        assert st["cg_its"][1] < st["cg_its"][0]
