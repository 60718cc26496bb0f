"""Sparse products on the GPU for the Schur-complement approximations of
Section 4 (eq. approx_positive_schur_general, C = 0): the CSR product and
transpose against SciPy on seeded matrices with ragged and empty rows, the
assembled -St = G M_bras^-1 G^T against the oracle's plain products, the
spectral bound of Lemma schur_condition_number_from_mass on the GPU's St,
reproducibility, and the error paths."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fe as ofe, mesh as omesh, assembly as oasm, schur as oschur, spectral
import workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(A):
    import torch
    A = sp.csr_matrix(A)
    A.sort_indices()
    return (torch.from_numpy(A.indptr.astype(np.int64)).cuda(), torch.from_numpy(A.indices.astype(np.int32)).cuda(),
            torch.from_numpy(A.data.astype(np.float64)).cuda())


def to_host(t, shape):
    rp, col, val = (x.cpu().numpy() for x in t)
    return sp.csr_matrix((val, col, rp), shape=shape)


def random_csr(m, n, max_row, seed, empty_every=7):
    """Ragged rows of 0..max_row distinct columns, every empty_every-th row empty."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(m):
        if i % empty_every == 3:
            continue
        c = rng.choice(n, size=rng.integers(1, max_row + 1), replace=False)
        rows += [i] * len(c)
        cols += list(c)
    vals = rng.uniform(-1.0, 1.0, len(rows))
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    A.sort_indices()
    return A


def same_pattern(X, Y):
    X, Y = sp.csr_matrix(X), sp.csr_matrix(Y)
    X.sort_indices()
    Y.sort_indices()
    return np.array_equal(X.indptr, Y.indptr) and np.array_equal(X.indices, Y.indices)


@pytest.mark.parametrize("m,k,n,ra,rb", [(1, 1, 1, 1, 1), (37, 53, 41, 5, 9), (300, 200, 500, 12, 30), (1000, 64, 3000, 3, 64)])
def test_spgemm_and_transpose_match_scipy(m, k, n, ra, rb):
    from paper_2607_12138_amd.problem import spgemm, csr_transpose
    A = random_csr(m, k, ra, 100 + m)
    B = random_csr(k, n, rb, 200 + k)
    say("spgemm %dx%d * %dx%d" % (m, k, k, n))
    Cg = to_host(spgemm(to_dev(A), to_dev(B), m, k), (m, n))
    # the pattern of all candidate products (no entry cancels in the symbolic product)
    Cpat = sp.csr_matrix((np.ones_like(A.data), A.indices, A.indptr), shape=A.shape) @ \
        sp.csr_matrix((np.ones_like(B.data), B.indices, B.indptr), shape=B.shape)
    assert same_pattern(Cg, Cpat)
    Cr = A @ B
    scale = (abs(A) @ abs(B)).toarray()
    assert np.all(np.abs((Cg - Cr).toarray()) <= 4 * 2.0 ** -52 * (ra + 1) * scale + 1e-300)
    say("transpose %dx%d" % (m, k))
    At = to_host(csr_transpose(to_dev(A), m, k), (k, m))
    Ar = A.T.tocsr()
    Ar.sort_indices()
    assert same_pattern(At, Ar) and np.array_equal(At.data, Ar.data)


SCHUR = [("P", 2, 2, 6, 0.2), ("N1curl", 3, 1, 3, 0.2), ("RT", 2, 2, 5, 0.2), ("BDM", 3, 1, 2, 0.0),
         ("P", 3, 3, 4, 0.2)]   # P3: 36 rows of (G M_bras^-1) G^T past 2048 candidates (the sort in HBM)


@pytest.mark.parametrize("case", SCHUR, ids=lambda c: "%s%d-%dd-N%d" % (c[0], c[2], c[1], c[3]))
def test_schur_matches_oracle_and_bound(case):
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import MassProblem
    family, dim, deg, N, jit = case
    coords, cells = omesh.structured_mesh(dim, N, jitter=jit, seed=4)
    orc = oasm.Problem(ofe.reference_element(family, dim, deg), coords, cells)
    gpu = MassProblem(family, dim, deg, N, jitter=jit, seed=4)
    # G: one row per element of a subset of the mesh, U[-1,1] on its DOFs
    m = min(len(orc.pi), orc.n // 2)
    rows = np.repeat(np.arange(m), orc.pi.shape[1])
    G = sp.csr_matrix((workloads.vector(rows.size, 9), (rows, orc.pi[:m].ravel())), shape=(m, orc.n))
    say("schur %s: G %dx%d" % (case, m, orc.n))
    St = to_host(gpu.schur(to_dev(G), L.OP_BRAS), (m, m))
    Sr = oschur.schur_approx(G, orc.B)
    scale = abs(G) @ abs(orc.B) @ abs(G).T
    assert same_pattern(St, scale)
    # each BRAS entry carries about 10 cond(M_K) eps relative error (both sides
    # invert M_K in their own order); the products sum entries of both signs
    kap_k = np.max(np.linalg.cond(orc.mats))
    tol = max(1e-13, 10 * kap_k * 2.0 ** -53)
    assert abs(St - Sr).max() <= tol * scale.max()
    # the lemma on the GPU's approximation: kappa(S_0, St_0) <= kappa(M, Mt)
    a0, b0 = oschur.generalized_extremes(St, oschur.exact_schur(G, orc.M))
    kap, lmin, lmax = spectral.kappa_hat(orc.M, orc.B)
    assert b0 / a0 <= kap * (1 + 1e-9)
    # the mass operator in place of its inverse: G M G^T, the same products
    Sm = to_host(gpu.schur(to_dev(G), L.OP_MASS), (m, m))
    Smr = G @ orc.M @ G.T
    assert abs(Sm - Smr).max() <= 1e-13 * (abs(G) @ abs(orc.M) @ abs(G).T).max()
    gpu.close()


def test_spgemm_is_reproducible_and_rejects_bad_input():
    import torch
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import spgemm
    A = random_csr(500, 300, 10, 7)
    B = random_csr(300, 800, 20, 8)
    a, b = to_dev(A), to_dev(B)
    c1 = spgemm(a, b, 500, 300)
    c2 = spgemm(a, b, 500, 300)
    assert all(torch.equal(x, y) for x, y in zip(c1, c2))
    rp = torch.empty(501, dtype=torch.int64, device="cuda")
    # a column of A outside the rows of B
    with pytest.raises(L.BrasError) as e:
        L.bras_spgemm_rowptr(500, 100, a, b, rp)          # A's columns reach 299
    assert e.value.code == L.BRAS_EINVAL
    # a column of A outside the rows of B past the entries the LDS route
    # scans (its first 64 entries already select 3840 candidates): the sort
    # in device memory validates the whole row
    W = sp.csr_matrix(np.ones((1, 100)))
    Wb = sp.csr_matrix(np.ones((100, 60)))
    with pytest.raises(L.BrasError) as e:
        L.bras_spgemm_rowptr(1, 99, to_dev(W), to_dev(Wb), torch.empty(2, dtype=torch.int64, device="cuda"))
    assert e.value.code == L.BRAS_EINVAL
    # row pointers of C that do not match the counts
    bad = (c1[0].clone(), c1[1].clone(), c1[2].clone())
    bad[0][1:] += 1
    with pytest.raises(L.BrasError):
        L.bras_spgemm_fill(500, 300, a, b, (bad[0], torch.empty(bad[1].numel() + 600, dtype=torch.int32, device="cuda"),
                                           torch.empty(bad[1].numel() + 600, dtype=torch.float64, device="cuda")))
    # a transpose with a column outside [0, n)
    from paper_2607_12138_amd.problem import csr_transpose
    with pytest.raises(L.BrasError):
        csr_transpose(a, 500, 250)
    torch.cuda.synchronize()


@pytest.mark.parametrize("m,n,ra,rb", [(1, 1, 1, 1), (50, 40, 6, 9), (800, 3000, 20, 5)])
def test_csr_add_matches_scipy(m, n, ra, rb):
    from paper_2607_12138_amd.problem import csr_add
    A = random_csr(m, n, ra, 300 + m)
    B = random_csr(m, n, rb, 400 + m, empty_every=5)
    say("csr add %dx%d" % (m, n))
    Cg = to_host(csr_add(to_dev(A), to_dev(B), m), (m, n))
    pat = abs(A) + abs(B)
    assert same_pattern(Cg, pat)
    # a + b is one rounding, as in SciPy: equal bit for bit
    Cr = (A + B).tocsr()
    Cr.sort_indices()
    Cg.sort_indices()
    assert np.array_equal(Cg.toarray(), Cr.toarray())


def test_schur_with_c_term_matches_oracle():
    """-St = C + G M_bras^-1 G^T with a sparse symmetric positive semi-definite C
    (the stabilisation block of eq. saddle_matrix_general_22), against the
    oracle and the C >= 0 bound of Lemma schur_condition_number_from_mass."""
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import MassProblem
    family, dim, deg, N, jit = "RT", 2, 2, 5, 0.2
    coords, cells = omesh.structured_mesh(dim, N, jitter=jit, seed=4)
    orc = oasm.Problem(ofe.reference_element(family, dim, deg), coords, cells)
    gpu = MassProblem(family, dim, deg, N, jitter=jit, seed=4)
    m = min(len(orc.pi), orc.n // 2)
    rows = np.repeat(np.arange(m), orc.pi.shape[1])
    G = sp.csr_matrix((workloads.vector(rows.size, 9), (rows, orc.pi[:m].ravel())), shape=(m, orc.n))
    H = sp.random(m, m // 3, density=0.05, random_state=np.random.default_rng(3), format="csr")
    Cm = (H @ H.T).tocsr()
    Cm.sort_indices()
    St = to_host(gpu.schur(to_dev(G), L.OP_BRAS, to_dev(Cm)), (m, m))
    Sr = oschur.schur_approx(G, orc.B, Cm)
    scale = abs(G) @ abs(orc.B) @ abs(G).T + abs(Cm)
    assert same_pattern(St, scale)
    kap_k = np.max(np.linalg.cond(orc.mats))
    assert abs(St - Sr).max() <= max(1e-13, 10 * kap_k * 2.0 ** -53) * scale.max()
    a0, b0 = oschur.alpha0_beta0(G, orc.M, orc.B)
    ac, bc = oschur.generalized_extremes(St, oschur.exact_schur(G, orc.M, Cm))
    assert bc / ac <= max(1.0, b0) / min(1.0, a0) * (1 + 1e-9)
    gpu.close()


@pytest.mark.parametrize("case", SCHUR[:3], ids=lambda c: "%s%d-%dd-N%d" % (c[0], c[2], c[1], c[3]))
def test_diagonal_schur_and_bras_comparison(case):
    """-St with diag(M)^-1 (the approximation BRAS is compared with in
    Section 4) against the oracle, and the BRAS St closer to S: its
    beta_0 / alpha_0 below the diagonal one, both from the GPU's products."""
    from paper_2607_12138_amd import _lib as L
    from paper_2607_12138_amd.problem import MassProblem
    family, dim, deg, N, jit = case
    coords, cells = omesh.structured_mesh(dim, N, jitter=jit, seed=4)
    orc = oasm.Problem(ofe.reference_element(family, dim, deg), coords, cells)
    gpu = MassProblem(family, dim, deg, N, jitter=jit, seed=4)
    D = gpu.assemble(L.OP_JACOBI)
    assert np.array_equal(D[0].cpu().numpy(), np.arange(orc.n + 1)) and np.array_equal(D[1].cpu().numpy(), np.arange(orc.n))
    assert np.max(np.abs(D[2].cpu().numpy() * orc.diag - 1.0)) <= 1e-14
    m = min(len(orc.pi), orc.n // 2)
    rows = np.repeat(np.arange(m), orc.pi.shape[1])
    G = sp.csr_matrix((workloads.vector(rows.size, 19), (rows, orc.pi[:m].ravel())), shape=(m, orc.n))
    Sd = to_host(gpu.schur(to_dev(G), L.OP_JACOBI), (m, m))
    Sdr = oschur.schur_approx(G, sp.diags(1.0 / orc.diag))
    scale = abs(G) @ sp.diags(1.0 / orc.diag) @ abs(G).T
    assert same_pattern(Sd, scale)
    assert abs(Sd - Sdr).max() <= 1e-13 * scale.max()
    Sb = to_host(gpu.schur(to_dev(G), L.OP_BRAS), (m, m))
    S = oschur.exact_schur(G, orc.M)
    ab, bb = oschur.generalized_extremes(Sb, S)
    ad, bd = oschur.generalized_extremes(Sd, S)
    say("  kappa(S, St): BRAS %.3f, diagonal %.3f" % (bb / ab, bd / ad))
    assert bb / ab < bd / ad
    gpu.close()


def ordered_product(A, B):
    """C = A B with each entry the sum of its products taken in the order of
    A's columns, then B's (the order the library documents), in float64."""
    A, B = sp.csr_matrix(A), sp.csr_matrix(B)
    A.sort_indices()
    B.sort_indices()
    rp, cols, vals = [0], [], []
    for i in range(A.shape[0]):
        acc = {}
        for p in range(A.indptr[i], A.indptr[i + 1]):
            a, av = A.indices[p], float(A.data[p])
            for q in range(B.indptr[a], B.indptr[a + 1]):
                j, v = int(B.indices[q]), av * float(B.data[q])
                acc[j] = acc[j] + v if j in acc else v
        ks = sorted(acc)
        cols += ks
        vals += [acc[j] for j in ks]
        rp.append(len(cols))
    return sp.csr_matrix((np.array(vals, dtype=np.float64), np.array(cols, dtype=np.int64), np.array(rp)),
                         shape=(A.shape[0], B.shape[1]))


def cap_case():
    """B (6000 x 4000): rows 0..1999 of 32 seeded columns, row 2999 of one,
    the rest empty.  Rows of A at and past the LDS variants' limits (1024
    and 2048 candidates or entries): 1024 candidates, 1056, 2048, 1509
    entries with 320 candidates, 2049 candidates, 2120 entries with 640
    candidates and the same row without its empty B rows, 2100 entries all
    selecting empty B rows, 22400 candidates, an empty row, a short row."""
    k, n = 6000, 4000
    rng = np.random.default_rng(17)
    brows = np.r_[np.repeat(np.arange(2000), 32), 2999]
    bcols = np.r_[np.concatenate([rng.choice(n, 32, replace=False) for _ in range(2000)]), 5]
    B = sp.csr_matrix((rng.uniform(-1, 1, brows.size), (brows, bcols)), shape=(k, n))
    B.sort_indices()
    sel = [np.arange(0, 32), np.arange(100, 133), np.arange(500, 564),
           np.r_[np.arange(10, 20), np.arange(2000, 2999), np.arange(3000, 3500)],
           np.r_[np.arange(600, 664), 2999],
           np.r_[np.arange(700, 720), np.arange(3000, 5100)],
           np.arange(700, 720),
           np.arange(3000, 5100),
           np.arange(1000, 1700),
           np.arange(0, 0),
           np.array([1, 2999])]
    arows = np.concatenate([np.full(len(x), i) for i, x in enumerate(sel)])
    acols = np.concatenate(sel)
    A = sp.csr_matrix((rng.uniform(-1, 1, arows.size), (arows, acols)), shape=(len(sel), k))
    A.sort_indices()
    # rows 5 and 6 select the same products in the same order
    A.data[A.indptr[6]:A.indptr[7]] = A.data[A.indptr[5]:A.indptr[5] + 20]
    return A, B, k, n


@pytest.mark.parametrize("shift", [0, 2095000, 4190400])
@pytest.mark.parametrize("lds_max", ["", "2048", "0"])
def test_spgemm_candidate_cap_boundaries(lds_max, shift, monkeypatch):
    """Rows at and past the LDS variants' limits against the candidate-order
    sums, bit for bit, with the default LDS limit (1024: the half-LDS variant
    and the sort in device memory), with 2048 (both LDS variants, the sort
    past 2048) and with 0 (every non-empty row sorted in device memory); a
    row whose extra entries select only empty B rows gives the same row as
    without them.  B's columns shifted up so that the LDS keys are 32-bit in
    both variants (0), 32-bit in the 1024 variant only (2095000: columns
    past 2^21) or 64-bit in both (4190400: columns past 2^22)."""
    from paper_2607_12138_amd.problem import spgemm
    A, B, k, n = cap_case()
    if shift:
        B = sp.csr_matrix((B.data, B.indices + shift, B.indptr), shape=(k, n + shift))
        n += shift
    if lds_max:
        monkeypatch.setenv("BRAS_SPGEMM_LDS_MAX", lds_max)
    bl = np.diff(B.indptr)
    cand = [int(bl[A.indices[A.indptr[i]:A.indptr[i + 1]]].sum()) for i in range(A.shape[0])]
    assert cand == [1024, 1056, 2048, 320, 2049, 640, 640, 0, 22400, 0, 33]
    say("spgemm at the candidate caps")
    Cg = to_host(spgemm(to_dev(A), to_dev(B), A.shape[0], k), (A.shape[0], n))
    Cr = ordered_product(A, B)
    assert np.array_equal(Cg.indptr, Cr.indptr) and np.array_equal(Cg.indices, Cr.indices)
    assert np.array_equal(Cg.data, Cr.data)
    assert Cg.indptr[8] == Cg.indptr[7]          # 2100 entries, no candidates
    assert np.array_equal(Cg.indices[Cg.indptr[5]:Cg.indptr[6]], Cg.indices[Cg.indptr[6]:Cg.indptr[7]])
    assert np.array_equal(Cg.data[Cg.indptr[5]:Cg.indptr[6]], Cg.data[Cg.indptr[6]:Cg.indptr[7]])
    if not shift:
        assert np.abs((Cg - A @ B).toarray()).max() <= 1e-13 * (abs(A) @ abs(B)).toarray().max()


@pytest.mark.parametrize("batch", ["1", "2100", "25000"])
def test_spgemm_long_rows_in_batches(batch, monkeypatch):
    """The sort in device memory split into batches of other sizes (one row
    each, several rows, all rows): the same product, bit for bit."""
    import torch
    from paper_2607_12138_amd.problem import spgemm
    A, B, k, n = cap_case()
    a, b = to_dev(A), to_dev(B)
    say("spgemm, long rows in batches of %s" % batch)
    ref = spgemm(a, b, A.shape[0], k)
    monkeypatch.setenv("BRAS_SPGEMM_BATCH", batch)
    got = spgemm(a, b, A.shape[0], k)
    monkeypatch.delenv("BRAS_SPGEMM_BATCH")
    assert all(torch.equal(x, y) for x, y in zip(ref, got))
