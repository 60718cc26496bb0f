"""Oracle pins for the Schur-complement approximations of Section 4: the
spectral bounds of Lemma schur_condition_number_from_mass hold for the BRAS
and the diagonal mass inverses, the exact inverse reproduces the exact Schur
complement, and the approximations are symmetric positive definite."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fe, mesh, assembly, spectral, schur
import workloads

CASES = [("P", 2, 2, 4, 0.2), ("N1curl", 3, 1, 2, 0.2), ("RT", 2, 2, 3, 0.2), ("BDM", 2, 1, 4, 0.0)]


def problem(case):
    family, dim, deg, N, jit = case
    coords, cells = mesh.structured_mesh(dim, N, jitter=jit, seed=3)
    return assembly.Problem(fe.reference_element(family, dim, deg), coords, cells)


def coupling(orc, seed):
    """G: one row per element of a subset of the mesh (fewer rows than DOFs),
    U[-1,1] values on the element's DOFs: full row rank with probability 1."""
    m = min(len(orc.pi), orc.n // 2)
    rows = np.repeat(np.arange(m), orc.pi.shape[1])
    vals = workloads.vector(rows.size, seed)
    return sp.csr_matrix((vals, (rows, orc.pi[:m].ravel())), shape=(m, orc.n))


def ids(c):
    return "%s%d-%dd-N%d" % (c[0], c[2], c[1], c[3])


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_schur_bound_from_mass_bound(case):
    """kappa_hat(S_0, St_0) = beta_0 / alpha_0 <= kappa_hat(M, Mt) (C = 0), and
    with C >= 0 the bound max(1, beta_0) / min(1, alpha_0) <= max(1, lmax) / min(1, lmin)."""
    orc = problem(case)
    G = coupling(orc, 11)
    for Minv in (orc.B, sp.diags(1.0 / orc.diag)):
        kap, lmin, lmax = spectral.kappa_hat(orc.M, Minv)
        a0, b0 = schur.alpha0_beta0(G, orc.M, Minv)
        assert a0 >= lmin * (1 - 1e-10) and b0 <= lmax * (1 + 1e-10)
        assert b0 / a0 <= kap * (1 + 1e-10)
        H = sp.csr_matrix(workloads.vector(G.shape[0] * 2, 12).reshape(G.shape[0], 2))
        C = H @ H.T                                          # symmetric positive semi-definite, rank 2
        S = schur.exact_schur(G, orc.M, C)
        St = schur.schur_approx(G, Minv, C).toarray()
        ac, bc = schur.generalized_extremes(St, S)
        assert bc / ac <= max(1.0, b0) / min(1.0, a0) * (1 + 1e-10)
        assert max(1.0, b0) / min(1.0, a0) <= max(1.0, lmax) / min(1.0, lmin) * (1 + 1e-10)
    # BRAS gives the tighter Schur bound on these meshes, as it gives the tighter mass bound
    kb = np.divide(*schur.alpha0_beta0(G, orc.M, orc.B)[::-1])
    kd = np.divide(*schur.alpha0_beta0(G, orc.M, sp.diags(1.0 / orc.diag))[::-1])
    assert kb < kd


@pytest.mark.parametrize("case", CASES[:2], ids=ids)
def test_exact_inverse_and_spd(case):
    orc = problem(case)
    G = coupling(orc, 21)
    Minv = np.linalg.inv(orc.M.toarray())
    S = schur.exact_schur(G, orc.M)
    assert np.allclose(schur.schur_approx(G, Minv).toarray(), S, rtol=0, atol=1e-12 * np.abs(S).max())
    a0, b0 = schur.alpha0_beta0(G, orc.M, Minv)
    assert abs(a0 - 1) < 1e-10 and abs(b0 - 1) < 1e-10
    St = schur.schur_approx(G, orc.B).toarray()
    assert np.array_equal(St, St.T) or np.abs(St - St.T).max() <= 1e-15 * np.abs(St).max()
    assert np.linalg.eigvalsh(0.5 * (St + St.T))[0] > 0


def test_bound_detects_a_wrong_operator():
    """A plausible mistake (M in place of an inverse of M) breaks the bound."""
    orc = problem(CASES[0])
    G = coupling(orc, 31)
    kap, lmin, lmax = spectral.kappa_hat(orc.M, orc.B)
    a0, b0 = schur.alpha0_beta0(G, orc.M, orc.M)
    assert b0 / a0 > kap
