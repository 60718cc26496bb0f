"""Pins for the oracle's BRAS operator against what the paper proves or prints."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fe, mesh, assembly, spectral, pcg
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def problem(family, dim, deg, N, jitter=0.0, seed=3, rho=None):
    ref = fe.reference_element(family, dim, deg)
    coords, cells = mesh.structured_mesh(dim, N, jitter=jitter, seed=seed)
    return assembly.Problem(ref, coords, cells, rho=rho)


SMALL = [("P", 2, 1, 4, 0.0), ("P", 2, 3, 3, 0.2), ("P", 3, 2, 2, 0.2), ("P", 3, 4, 1, 0.0),
         ("N1curl", 3, 2, 2, 0.2), ("RT", 3, 2, 2, 0.2), ("RT", 2, 2, 3, 0.2), ("N1curl", 2, 3, 2, 0.2)]


@pytest.mark.parametrize("family,dim,deg,N,jit", SMALL)
def test_bras_symmetric_positive_definite(family, dim, deg, N, jit):
    pr = problem(family, dim, deg, N, jit)
    B = pr.B.toarray()
    assert np.max(np.abs(B - B.T)) <= 1e-13 * np.max(np.abs(B))
    np.linalg.cholesky(B)                         # SPD (eq. mhatinvbras_def, full-rank P)
    # nonzeros only between DOFs that share an element: the element-adjacency
    # graph of M (eq. mass_and_bras_element_sums)
    inc = sp.csr_matrix((np.ones(pr.pi.size), (pr.pi.ravel(), np.repeat(np.arange(len(pr.pi)), pr.pi.shape[1]))),
                        shape=(pr.n, len(pr.pi)))
    adj = (inc @ inc.T).tocsr()
    adj_set = set(zip(*adj.nonzero()))
    assert set(zip(*pr.B.nonzero())) <= adj_set
    assert set(zip(*pr.M.nonzero())) <= adj_set


@pytest.mark.parametrize("family,dim,deg,N,jit", SMALL)
def test_lambda_min_at_least_one(family, dim, deg, N, jit):
    # Cor. bras_lambda_min
    pr = problem(family, dim, deg, N, jit)
    ev = spectral.preconditioned_eigs(pr.M, pr.B)
    assert ev[0] >= 1.0 - 1e-10


@pytest.mark.parametrize("family,dim,deg,N", [("RT", 3, 1, 2), ("RT", 3, 2, 2), ("RT", 2, 2, 3)])
def test_lambda_min_equals_one_when_nbr_below_2n(family, dim, deg, N):
    pr = problem(family, dim, deg, N, 0.2)
    assert pr.n_br < 2 * pr.n                     # sum_i (d_i - 2) < 0
    assert np.sum(pr.d - 2) == pr.n_br - 2 * pr.n
    ev = spectral.preconditioned_eigs(pr.M, pr.B)
    assert abs(ev[0] - 1.0) < 1e-10


@pytest.mark.parametrize("dim,deg,N", [(2, 1, 8), (3, 1, 3), (2, 2, 4), (2, 3, 3), (3, 3, 2), (3, 4, 1)])
def test_constant_is_fixed_on_uniform_meshes(dim, deg, N):
    # M_br P 1 in range(P) on equal-volume meshes => Mbras^-1 M 1 = 1
    pr = problem("P", dim, deg, N)
    one = np.ones(pr.n)
    y = pr.B @ (pr.M @ one)
    assert np.max(np.abs(y - 1.0)) < 1e-13


def test_constant_not_fixed_on_jittered_mesh():
    pr = problem("P", 2, 1, 6, 0.2)
    y = pr.B @ (pr.M @ np.ones(pr.n))
    assert np.max(np.abs(y - 1.0)) > 1e-3


@pytest.mark.parametrize("family,dim,deg,N,jit", SMALL[:6])
def test_lambda_max_projector_identity(family, dim, deg, N, jit):
    # Thm. bras_lambda_max_projector
    pr = problem(family, dim, deg, N, jit)
    lmax = spectral.preconditioned_eigs(pr.M, pr.B)[-1]
    lq = spectral.projector_lambda_max(pr.pi, pr.mats, pr.n)
    assert abs(lmax - lq) < 1e-10 * lmax


@pytest.mark.parametrize("family,dim,deg,N,jit", [("P", 2, 2, 2, 0.2), ("N1curl", 3, 1, 1, 0.0), ("RT", 2, 2, 2, 0.2), ("P", 3, 1, 2, 0.2)])
def test_exact_inverse_correction(family, dim, deg, N, jit):
    # Lemma bras_exact_inverse_correction: Mbras^-1 = M^-1 - Z S^-1 Z^T, correction SPSD
    pr = problem(family, dim, deg, N, jit)
    rhs, corr = spectral.exact_inverse_correction(pr.pi, pr.mats, pr.n)
    B = pr.B.toarray()
    assert np.max(np.abs(B - rhs)) < 1e-10 * np.max(np.abs(B))
    assert np.linalg.eigvalsh(0.5 * (corr + corr.T))[0] > -1e-10 * np.max(np.abs(corr))


@pytest.mark.parametrize("family,deg", [("P", 2), ("N1curl", 2), ("RT", 2)])
def test_metric_contrast_bound(family, deg):
    # Cor. bras_piola_metric_contrast: lambda_max(B^G M^G) <= beta/alpha lambda_max(B^I M^I)
    ref = fe.reference_element(family, 3, deg)
    coords, cells = mesh.structured_mesh(3, 2, jitter=0.2, seed=21)
    prG = assembly.Problem(ref, coords, cells)
    G = assembly.metric(family, coords, cells)
    ratio = spectral.metric_contrast(family, G)
    mI = ref.mass if family == "P" else sum(ref.mass[a, a] for a in range(3))
    matsI = np.broadcast_to(mI, (len(cells),) + mI.shape).copy()
    MI = assembly.mass_matrix(prG.pi, matsI, prG.n)
    BI = assembly.bras_matrix(prG.pi, matsI, prG.n, prG.d)
    lG = spectral.preconditioned_eigs(prG.M, prG.B)[-1]
    lI = spectral.preconditioned_eigs(MI, BI)[-1]
    assert lG <= ratio * lI * (1 + 1e-10)
    assert ratio > 1.0


@pytest.mark.parametrize("family,dim,deg", [("P", 3, 3), ("RT", 3, 2), ("N1curl", 3, 2), ("P", 2, 4)])
def test_single_element_is_exact(family, dim, deg):
    ref = fe.reference_element(family, dim, deg)
    coords, cells = mesh.structured_mesh(dim, 1, jitter=0.0)
    coords = coords[cells[0]]
    cells = np.arange(dim + 1, dtype=np.int32)[None, :]
    pr = assembly.Problem(ref, coords, cells)
    assert np.all(pr.d == 1)
    B = pr.B.toarray()
    M = pr.M.toarray()
    assert np.max(np.abs(B @ M - np.eye(pr.n))) < 1e-11


def test_broken_map_gives_one_iteration():
    # P = I (every d_i = 1): Mbras^-1 = M^-1 and PCG stops after one product
    ref = fe.reference_element("P", 2, 2)
    coords, cells = mesh.structured_mesh(2, 3, jitter=0.2, seed=1)
    mats = assembly.element_matrices(ref, coords, cells)
    pi = np.arange(len(cells) * ref.n_loc).reshape(len(cells), ref.n_loc)
    n = pi.size
    M = assembly.mass_matrix(pi, mats, n)
    B = assembly.bras_matrix(pi, mats, n)
    b = workloads.vector(n, 5)
    x, its, ok, _ = pcg.pcg(M, b, B.dot, tol=1e-12)
    assert ok and its == 1


@pytest.mark.parametrize("family,dim,deg,N,jit,R", [("P", 3, 3, 2, 0.2, 1), ("RT", 3, 2, 2, 0.2, 3), ("N1curl", 3, 2, 2, 0.2, 1)])
def test_matrix_free_routes_agree(family, dim, deg, N, jit, R):
    pr = problem(family, dim, deg, N, jit)
    x = workloads.rhs(pr.n, R, 9)
    inv = assembly.element_inverses(pr.mats)
    y1 = assembly.bras_apply_matrix_free(pr.pi, inv, pr.d, x)
    y2 = pr.B @ x
    assert np.max(np.abs(y1 - y2)) <= 1e-13 * np.max(np.abs(y2))
    if R == 1:
        m1 = assembly.mass_apply_matrix_free(pr.pi, pr.mats, x)
        m2 = pr.M @ x
        assert np.max(np.abs(m1 - m2)) <= 1e-13 * np.max(np.abs(m2))
    # assembly identity M = P^T Mbr P as a sparse triple product
    P = spectral.injection(pr.pi, pr.n)
    Mt = (P.T @ spectral.broken_mass(pr.mats) @ P).toarray()
    assert np.max(np.abs(Mt - pr.M.toarray())) <= 1e-14 * np.max(np.abs(Mt))


def test_diagonal_scaling_invariance():
    # A diagonal change of basis S leaves kappa-hat of both preconditioners unchanged
    pr = problem("RT", 3, 2, 1, 0.2)
    s = np.linspace(0.5, 2.0, pr.n)
    S = sp.diags(s)
    mats_s = pr.mats * s[pr.pi][:, :, None] * s[pr.pi][:, None, :]
    Ms = assembly.mass_matrix(pr.pi, mats_s, pr.n)
    Bs = assembly.bras_matrix(pr.pi, mats_s, pr.n, pr.d)
    assert np.max(np.abs((S @ pr.M @ S - Ms).toarray())) < 1e-13 * abs(Ms).max()
    k1 = spectral.kappa_hat(pr.M, pr.B)[0]
    k2 = spectral.kappa_hat(Ms, Bs)[0]
    assert abs(k1 - k2) < 1e-9 * k1


def _entity_blocks(ref):
    """Local DOF ranges of each entity (vertices, edges, faces, interior), in local order."""
    import itertools
    d = ref.dim
    out, o = [], 0
    for edim, cnt in enumerate(ref.dofs_per_entity):
        for _ in itertools.combinations(range(d + 1), edim + 1):
            out.append((edim, o, o + cnt))
            o += cnt
    assert o == ref.n_loc
    return out


@pytest.mark.parametrize("family,dim,deg,N", [("N1curl", 3, 3, 1), ("RT", 3, 3, 1), ("P", 2, 4, 2),
                                              ("N1curl", 2, 3, 2)])
def test_bras_spectrum_invariant_under_entity_basis_change(family, dim, deg, N):
    """Recombining the basis functions of each mesh entity (the same invertible
    map T_e for every cell sharing the entity) changes M to S^T M S with S
    entity-block diagonal; d is constant on an entity, so D^-1 commutes with S
    and Mbras^-1 M becomes S^-1 (Mbras^-1 M) S: the BRAS spectrum depends only
    on the span of each entity's functions, not on the moment variant, while
    the diagonal preconditioner's spectrum does depend on it."""
    pr = problem(family, dim, deg, N, 0.2)
    g = np.random.default_rng(5)
    S = np.zeros((pr.ref.n_loc, pr.ref.n_loc))
    T = {}
    for edim, a, b in _entity_blocks(pr.ref):
        if b > a:
            # one map per entity dimension; it is the same for every edge (face) of
            # every cell because local entity DOFs follow the sorted-vertex order
            T.setdefault(edim, np.eye(b - a) + 0.5 * g.standard_normal((b - a, b - a)))
            S[a:b, a:b] = T[edim]
    mats_s = np.einsum("ji,kjl,lm->kim", S, pr.mats, S)
    Ms = assembly.mass_matrix(pr.pi, mats_s, pr.n)
    Bs = assembly.bras_matrix(pr.pi, mats_s, pr.n, pr.d)
    kb, kbs = spectral.kappa_hat(pr.M, pr.B)[0], spectral.kappa_hat(Ms, Bs)[0]
    kd = spectral.kappa_hat(pr.M, sp.diags(1.0 / pr.diag))[0]
    kds = spectral.kappa_hat(Ms, sp.diags(1.0 / Ms.diagonal()))[0]
    assert abs(kb - kbs) < 1e-8 * kb
    assert abs(kd - kds) > 1e-3 * kd


def _sig2(x):
    return float("%.2g" % x)


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "paper_kappa.json")))["cases"],
                         ids=lambda c: c["cite"])
def test_kappa_matches_paper_tables(case):
    pr = problem(case["family"], case["dim"], case["degree"], case["N"])
    assert 2000 <= pr.n <= 7500                  # "approximately 5e3 DOFs" (the closest Kuhn mesh)
    kb = spectral.kappa_hat(pr.M, pr.B)[0]
    assert _sig2(kb) == case["kappa_bras"], (kb, case)
    if case["kappa_diag"] is not None:
        kd = spectral.kappa_hat(pr.M, sp.diags(1.0 / pr.diag))[0]
        assert _sig2(kd) == case["kappa_diag"], (kd, case)


def test_two_dimensional_curl_and_div_are_rotations():
    # 2D N1curl_k and RT_k differ by a rotation: identical spectra (Tables hcurl/hdiv, 2D rows)
    for k in (1, 2):
        a = problem("N1curl", 2, k, 3, 0.2)
        b = problem("RT", 2, k, 3, 0.2)
        ka = spectral.kappa_hat(a.M, a.B)[0]
        kb = spectral.kappa_hat(b.M, b.B)[0]
        kda = spectral.kappa_hat(a.M, sp.diags(1.0 / a.diag))[0]
        kdb = spectral.kappa_hat(b.M, sp.diags(1.0 / b.diag))[0]
        assert abs(ka - kb) < 1e-9 * ka and abs(kda - kdb) < 1e-9 * kda


@pytest.mark.parametrize("family,dim,deg,N,R", [("P", 3, 3, 3, 1), ("N1curl", 3, 2, 2, 1), ("RT", 3, 2, 2, 3), ("P", 2, 4, 5, 2)])
def test_operator_rows_one_by_one(family, dim, deg, N, R):
    # row-by-row element sums (used for sampled checks at full size) agree with
    # the assembled matrices
    ref = fe.reference_element(family, dim, deg)
    coords, cells = mesh.structured_mesh(dim, N, jitter=0.2, seed=2)
    rho = workloads.density(len(cells), 3)
    pr = assembly.Problem(ref, coords, cells, rho=rho)
    x = workloads.rhs(pr.n, R, 3)
    rows = workloads.sample(pr.n, 12, 4)
    for which, A in (("mass", pr.M), ("bras", pr.B)):
        got = assembly.operator_rows(ref, coords, cells, pr.pi, pr.n, rows, x, which, rho=rho)
        want = (A @ x)[rows]
        assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(A @ x))


def test_gram_factor_identity_and_bf16_emulation_error():
    from oracle import reduced
    pr = problem("RT", 3, 2, 2, 0.2)
    G = reduced.gram_factors(pr.mats, pr.pi, pr.d)
    # G^T G = D_K^-1 M_K^-1 D_K^-1: the factor form reproduces BRAS exactly in float64
    x = workloads.rhs(pr.n, 2, 8)
    Z = np.einsum("kji,kjr->kir", G, np.einsum("kij,kjr->kir", G, x[pr.pi]))
    y = np.zeros_like(x)
    np.add.at(y, pr.pi.ravel(), Z.reshape(-1, 2))
    assert np.max(np.abs(y - pr.B @ x)) <= 1e-13 * np.max(np.abs(pr.B @ x))
    # BF16 emulation: error of order 2^-8 relative, and r^T B_bf16 r > 0
    yb = reduced.bras_apply_bf16_emulated(pr.pi, pr.mats, pr.d, x)
    err = np.max(np.abs(yb - pr.B @ x)) / np.max(np.abs(pr.B @ x))
    assert 1e-5 < err < 3e-2
    for r in range(2):
        assert x[:, r] @ yb[:, r] > 0
    assert reduced.round_bf16(np.array([1.0 + 2.0 ** -9]))[0] == 1.0          # tie to even
    assert reduced.round_bf16(np.array([1.0 + 3 * 2.0 ** -9]))[0] == 1.0 + 2.0 ** -7


@pytest.mark.parametrize("deg,N", [(1, 6), (3, 3)])
def test_rotated_stretch_bound(deg, N):
    """Eq. rot_stretch_map on a 2D BDM mesh: the map has det 1 and singular
    values r, 1/r, so relative to the unstretched mesh the H(div) metric has
    contrast r^4; lambda_min(Mbras^-1 M) stays 1 and Cor.
    bras_piola_metric_contrast bounds lambda_max by r^4 times the unstretched
    value.  BRAS stays below the diagonal preconditioner."""
    ref = fe.reference_element("BDM", 2, deg)
    coords, cells = mesh.structured_mesh(2, N, jitter=0.0, seed=0)
    base = assembly.Problem(ref, coords, cells)
    kb1, lo1, hi1 = spectral.kappa_hat(base.M, base.B)
    assert abs(lo1 - 1.0) < 1e-10
    for r in (3.0, 5.0):
        st = assembly.Problem(ref, workloads.rotated_stretch(coords, r), cells)
        J = mesh.jacobians(st.coords, cells)
        assert np.allclose(np.linalg.det(J), np.linalg.det(mesh.jacobians(coords, cells)), rtol=1e-12)
        kb, lo, hi = spectral.kappa_hat(st.M, st.B)
        kd = spectral.kappa_hat(st.M, sp.diags(1.0 / st.diag))[0]
        assert abs(lo - 1.0) < 1e-10
        assert hi <= r ** 4 * hi1 * (1 + 1e-12)
        assert hi > hi1                                  # the stretch does cost something
        assert kb < kd
