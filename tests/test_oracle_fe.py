"""Pins for the oracle's reference elements and element matrices."""
import itertools

import numpy as np
import pytest

from oracle import fe, mesh, dofmap, assembly
from tests.quadrature import simplex_rule, gauss01, orthonormal_numeric, moment_fields_numeric

ELEMENTS = [("P", 2, 1), ("P", 2, 2), ("P", 2, 3), ("P", 2, 4), ("P", 3, 1), ("P", 3, 2),
            ("P", 3, 3), ("P", 3, 4), ("RT", 2, 1), ("RT", 2, 3), ("N1curl", 2, 2),
            ("RT", 3, 1), ("RT", 3, 2), ("RT", 3, 4), ("N1curl", 3, 1), ("N1curl", 3, 2),
            ("N1curl", 3, 3), ("B", 2, 2), ("B", 2, 4), ("B", 3, 3), ("B", 3, 4),
            ("N2curl", 2, 1), ("N2curl", 2, 3), ("BDM", 2, 2), ("N2curl", 3, 1), ("N2curl", 3, 2),
            ("N2curl", 3, 3), ("BDM", 3, 1), ("BDM", 3, 2), ("BDM", 3, 3)]
SECOND_KIND = ("N2curl", "BDM")


def ref_volume(d):
    return 0.5 if d == 2 else 1.0 / 6.0


def test_p1_closed_forms():
    for d, den in ((2, 12.0), (3, 20.0)):
        e = fe.reference_element("P", d, 1)
        vol = ref_volume(d)
        expect = vol / den * (np.ones((d + 1, d + 1)) + np.eye(d + 1))
        assert np.allclose(e.mass, expect, rtol=0, atol=1e-16)
        # closed-form inverse (d+1)/|K| ((d+2) I - J) for a physical element
        scale = 0.37
        Minv = np.linalg.inv(scale * e.mass)
        expect_inv = (d + 1) / (scale * vol) * ((d + 2) * np.eye(d + 1) - np.ones((d + 1, d + 1)))
        assert np.allclose(Minv, expect_inv, rtol=1e-13, atol=0)


def test_gll_points_against_legendre_roots():
    for n in (2, 3, 4, 5, 6):
        g = fe.gll01(n)
        r = np.sort(np.polynomial.legendre.Legendre.basis(n).deriv().roots().real)
        assert np.allclose(g[1:-1], (r + 1) / 2, atol=1e-15)
        assert g[0] == 0.0 and g[-1] == 1.0


@pytest.mark.parametrize("d,p", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3), (3, 4)])
def test_lagrange_nodal_and_partition_of_unity(d, p):
    e = fe.reference_element("P", d, p)
    vals = e.eval(e.nodes)[:, :, 0]
    assert np.allclose(vals, np.eye(e.n_loc), atol=1e-12)
    pts, _ = simplex_rule(d, 5)
    assert np.allclose(e.eval(pts)[:, :, 0].sum(axis=1), 1.0, atol=1e-12)
    assert abs(e.mass.sum() - ref_volume(d)) < 1e-14 * ref_volume(d)
    # nodes lie on the entities they belong to: edge nodes are GLL points
    if p >= 2:
        g = fe.gll01(p)[1:-1]
        first_edge = e.nodes[d + 1:d + 1 + (p - 1)]
        # local edge (0,1): x = s e_1 with s ascending from vertex 0
        assert np.allclose(first_edge[:, 0], g, atol=1e-15)
        assert np.allclose(first_edge[:, 1:], 0.0, atol=1e-15)


def test_p4_face_nodes_are_symmetric_orbit():
    e = fe.reference_element("P", 3, 4)
    face0 = e.nodes[4 + 6 * 3:4 + 6 * 3 + 3]     # face (0,1,2): z = 0
    assert np.allclose(face0[:, 2], 0.0)
    bary = np.column_stack([1 - face0[:, 0] - face0[:, 1], face0[:, 0], face0[:, 1]])
    # an S3 orbit (a, a, 1-2a), node t nearest to face vertex t
    for t in range(3):
        assert np.argmax(bary[t]) == t
    assert np.allclose(np.sort(bary, axis=1), np.sort(bary[0])[None, :])
    assert np.allclose(e.nodes[-1], [0.25, 0.25, 0.25])


@pytest.mark.parametrize("family,d,k", ELEMENTS)
def test_mass_against_quadrature(family, d, k):
    e = fe.reference_element(family, d, k)
    pts, wts = simplex_rule(d, k + 2)
    phi = e.eval(pts)                         # [npts, n, c]
    if e.ncomp == 1:
        Mq = np.einsum("p,pi,pj->ij", wts, phi[:, :, 0], phi[:, :, 0])
        ref = e.mass
    else:
        Mq = np.einsum("p,pia,pjb->abij", wts, phi, phi)
        ref = e.mass
    assert np.max(np.abs(Mq - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("d,p", [(2, 3), (2, 4), (3, 3), (3, 4)])
def test_lagrange_polynomial_exactness(d, p):
    e = fe.reference_element("P", d, p)
    rng = np.random.default_rng(3)
    exps = [a for a in itertools.product(range(p + 1), repeat=d) if sum(a) <= p]
    cf, cg = rng.standard_normal(len(exps)), rng.standard_normal(len(exps))

    def poly(c, x):
        return sum(ci * np.prod(x ** np.array(a), axis=1) for ci, a in zip(c, exps))
    fv, gv = poly(cf, e.nodes), poly(cg, e.nodes)
    pts, wts = simplex_rule(d, p + 2)
    exact = np.sum(wts * poly(cf, pts) * poly(cg, pts))
    assert abs(fv @ e.mass @ gv - exact) < 1e-13 * max(1.0, abs(exact))


def _second_kind_functionals_numeric(family, d, k):
    rv = np.array(fe.ref_vertices(d), dtype=float)
    funcs = []
    if d == 2 or family == "N2curl":
        s, w = gauss01(k + 3)
        q = orthonormal_numeric(1, k)(s[:, None])
        for a, b in itertools.combinations(range(d + 1), 2):
            t = rv[b] - rv[a]
            dirv = t if family == "N2curl" else np.array([t[1], -t[0]])
            x = rv[a] + s[:, None] * t
            for m in range(q.shape[1]):
                funcs.append(lambda u, x=x, dirv=dirv, qm=q[:, m], w=w: np.sum(w * (u(x) @ dirv) * qm))
    if d == 3:
        st, w = simplex_rule(2, k + 3)
        for a, b, c in itertools.combinations(range(4), 3):
            t1, t2 = rv[b] - rv[a], rv[c] - rv[a]
            x = rv[a] + st[:, :1] * t1 + st[:, 1:] * t2
            if family == "BDM":
                q = orthonormal_numeric(2, k)(st)
                nrm = np.cross(t1, t2)
                for m in range(q.shape[1]):
                    funcs.append(lambda u, x=x, nv=nrm, qm=q[:, m], w=w: np.sum(w * (u(x) @ nv) * qm))
            elif k >= 2:
                F = moment_fields_numeric("RT", 2, k - 1)(st)              # [npts, nf, 2]
                T = np.stack([t1, t2])                                   # [2, 3]
                for m in range(F.shape[1]):
                    funcs.append(lambda u, x=x, T=T, Fm=F[:, m, :], w=w:
                                 np.sum(w * np.sum((u(x) @ T.T) * Fm, axis=1)))
    j = k - 1 if (family == "BDM" or d == 2) else k - 2
    ev = moment_fields_numeric("RT" if family == "N2curl" else "N1curl", d, j)
    if ev is not None:
        pts, w = simplex_rule(d, k + 3)
        F = ev(pts)
        for m in range(F.shape[1]):
            funcs.append(lambda u, pts=pts, Fm=F[:, m, :], w=w: np.sum(w * np.sum(u(pts) * Fm, axis=1)))
    return funcs


def _entity_functionals_numeric(family, d, k):
    """The moment functionals, evaluated by quadrature, as callables on a field
    function u(x) -> [npts, d] (independent of the oracle's exact route)."""
    if family in SECOND_KIND:
        return _second_kind_functionals_numeric(family, d, k)
    rv = np.array(fe.ref_vertices(d), dtype=float)
    funcs = []
    if family == "N1curl" or (family == "RT" and d == 2):
        s, w = gauss01(k + 3)
        q = orthonormal_numeric(1, k - 1)(s[:, None])
        for a, b in itertools.combinations(range(d + 1), 2):
            t = rv[b] - rv[a]
            dirv = t if family == "N1curl" else np.array([t[1], -t[0]])
            x = rv[a] + s[:, None] * t
            for m in range(q.shape[1]):
                funcs.append(lambda u, x=x, dirv=dirv, qm=q[:, m], w=w: np.sum(w * (u(x) @ dirv) * qm))
    if d == 3:
        st, w = simplex_rule(2, k + 3)
        for a, b, c in itertools.combinations(range(4), 3):
            t1, t2 = rv[b] - rv[a], rv[c] - rv[a]
            x = rv[a] + st[:, :1] * t1 + st[:, 1:] * t2
            if family == "RT":
                q = orthonormal_numeric(2, k - 1)(st)
                nrm = np.cross(t1, t2)
                for m in range(q.shape[1]):
                    funcs.append(lambda u, x=x, nv=nrm, qm=q[:, m], w=w: np.sum(w * (u(x) @ nv) * qm))
            elif k >= 2:
                q = orthonormal_numeric(2, k - 2)(st)
                for tt in (t1, t2):
                    for m in range(q.shape[1]):
                        funcs.append(lambda u, x=x, tv=tt, qm=q[:, m], w=w: np.sum(w * (u(x) @ tv) * qm))
    qdeg = k - 2 if (family == "RT" or d == 2) else k - 3
    if qdeg >= 0:
        pts, w = simplex_rule(d, k + 3)
        q = orthonormal_numeric(d, qdeg)(pts)
        for comp in range(d):
            for m in range(q.shape[1]):
                funcs.append(lambda u, pts=pts, comp=comp, qm=q[:, m], w=w: np.sum(w * u(pts)[:, comp] * qm))
    return funcs


@pytest.mark.parametrize("family,d,k", [el for el in ELEMENTS if el[0] not in ("P", "B")])
def test_vector_duality_numeric(family, d, k):
    e = fe.reference_element(family, d, k)
    funcs = _entity_functionals_numeric(family, d, k)
    assert len(funcs) == e.n_loc == fe.element_dim(family, d, k)
    A = np.array([[f(lambda x, j=j: e.eval(x)[:, j, :]) for j in range(e.n_loc)] for f in funcs])
    assert np.allclose(A, np.eye(e.n_loc), atol=1e-12)


@pytest.mark.parametrize("family,d,k", [el for el in ELEMENTS if el[0] not in ("P", "B")])
def test_vector_traces_and_field_reproduction(family, d, k):
    e = fe.reference_element(family, d, k)
    rng = np.random.default_rng(11)
    pts, wts = simplex_rule(d, k + 2)
    Phi = e.eval(pts)
    # a constant and a linear field of the space are reproduced exactly
    v = rng.standard_normal(d)
    fields = [lambda x: np.tile(v, (len(x), 1))]
    if family in SECOND_KIND:
        A = rng.standard_normal((d, d))
        fields.append(lambda x: x @ A.T)                        # any linear field is in [P_1]^d
    elif family == "RT":
        fields.append(lambda x: x.copy())                       # x in RT_1
    elif d == 3:
        fields.append(lambda x: np.cross(v, x))                 # v x x in N1curl_1
    else:
        fields.append(lambda x: np.stack([-x[:, 1], x[:, 0]], axis=1))
    Mid = sum(e.mass[a, a] for a in range(d))
    for f in fields:
        F = f(pts)
        c, *_ = np.linalg.lstsq(Phi.transpose(0, 2, 1).reshape(-1, e.n_loc), F.ravel(), rcond=None)
        assert np.allclose(np.einsum("pjc,j->pc", Phi, c), F, atol=1e-11)
        assert abs(c @ Mid @ c - np.sum(wts * np.sum(F * F, axis=1))) < 1e-12
    # normal (RT, BDM) / tangential (N1curl, N2curl) traces on an entity are in
    # P_{k-1} (first kind) or P_k (second kind)
    tdeg = k if family in SECOND_KIND else k - 1
    curl = family in ("N1curl", "N2curl")
    s = np.linspace(0.05, 0.95, 3 * k + 4)
    if curl or d == 2:
        t = np.zeros(d); t[0] = 1.0
        x = s[:, None] * t[None, :]
        dirv = t if curl else np.array([t[1], -t[0]])
        tr = e.eval(x) @ dirv
        Vd = np.vander(s, tdeg + 1, increasing=True)
        res = tr - Vd @ np.linalg.lstsq(Vd, tr, rcond=None)[0]
        assert np.max(np.abs(res)) < 1e-10
    if not curl and d == 3:
        st = rng.uniform(0, 0.5, size=(40, 2))
        x = np.column_stack([st, np.zeros(40)])               # face (0,1,2)
        tr = e.eval(x)[:, :, 2]
        ex = [a for a in itertools.product(range(tdeg + 1), repeat=2) if sum(a) <= tdeg]
        Vd = np.stack([st[:, 0] ** a * st[:, 1] ** b for a, b in ex], axis=1)
        res = tr - Vd @ np.linalg.lstsq(Vd, tr, rcond=None)[0]
        assert np.max(np.abs(res)) < 1e-9


def _pullback_dofs(family, ref, J, x0, f, d):
    """Broken DOFs of the global field f on one cell: reference functionals of
    the Piola pull-back (covariant: J^T f(F(xh)); contravariant: det J J^-1 f)."""
    funcs = _entity_functionals_numeric(family, d, ref.degree)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    if family in ("N1curl", "N2curl"):
        fh = lambda xh: f(x0 + xh @ J.T) @ J
    else:
        fh = lambda xh: det * (f(x0 + xh @ J.T) @ Jinv.T)
    return np.array([fn(fh) for fn in funcs])


@pytest.mark.parametrize("family,d,k", [("RT", 3, 2), ("N1curl", 3, 2), ("RT", 2, 2), ("N1curl", 2, 2), ("RT", 3, 1),
                                        ("BDM", 3, 1), ("BDM", 3, 2), ("N2curl", 3, 1), ("N2curl", 3, 2),
                                        ("N2curl", 2, 1), ("BDM", 2, 2)])
def test_global_conformity_and_l2_norm(family, d, k):
    ref = fe.reference_element(family, d, k)
    coords, cells = mesh.structured_mesh(d, 2, jitter=0.2, seed=5)
    pr = assembly.Problem(ref, coords, cells, need_bras=False)
    A = np.array([[0.3, -1.1, 0.4], [0.7, 0.2, -0.5], [0.1, 0.9, 0.6]])[:d, :d]
    c = np.array([0.5, -0.25, 1.0])[:d]
    f = lambda x: x @ A.T + c                                   # linear field: in both spaces for k >= 2
    if k == 1 and family not in SECOND_KIND:
        if family == "RT":
            f = lambda x: 0.7 * x + c
        else:
            f = lambda x: c
    Js = mesh.jacobians(coords, cells)
    w = np.array([_pullback_dofs(family, ref, Js[K], coords[cells[K, 0]], f, d) for K in range(len(cells))])
    u = np.zeros(pr.n)
    u[pr.pi.ravel()] = w.ravel()
    # every broken copy of a conforming DOF carries the same value
    assert np.max(np.abs(w - u[pr.pi])) < 1e-12
    pts, wts = simplex_rule(d, k + 2)
    tot = 0.0
    for K in range(len(cells)):
        x = coords[cells[K, 0]] + pts @ Js[K].T
        tot += abs(np.linalg.det(Js[K])) * np.sum(wts * np.sum(f(x) ** 2, axis=1))
    assert abs(u @ (pr.M @ u) - tot) < 1e-12 * tot


def test_h1_global_interpolant_l2_norm():
    ref = fe.reference_element("P", 3, 3)
    coords, cells = mesh.structured_mesh(3, 2, jitter=0.2, seed=4)
    pr = assembly.Problem(ref, coords, cells, need_bras=False)
    f = lambda x: 1.0 + x[:, 0] ** 3 - 2 * x[:, 0] * x[:, 1] * x[:, 2] + 0.5 * x[:, 2] ** 2
    Js = mesh.jacobians(coords, cells)
    w = np.array([f(coords[cells[K, 0]] + ref.nodes @ Js[K].T) for K in range(len(cells))])
    u = np.zeros(pr.n)
    u[pr.pi.ravel()] = w.ravel()
    assert np.max(np.abs(w - u[pr.pi])) < 1e-13
    pts, wts = simplex_rule(3, 5)
    tot = sum(abs(np.linalg.det(Js[K])) * np.sum(wts * f(coords[cells[K, 0]] + pts @ Js[K].T) ** 2)
              for K in range(len(cells)))
    assert abs(u @ (pr.M @ u) - tot) < 1e-13 * tot


@pytest.mark.parametrize("family", ["N1curl", "RT", "N2curl", "BDM"])
def test_piola_element_matrix_against_physical_quadrature(family):
    ref = fe.reference_element(family, 3, 2)
    coords, cells = mesh.structured_mesh(3, 2, jitter=0.2, seed=8)
    mats = assembly.element_matrices(ref, coords, cells)
    Js = mesh.jacobians(coords, cells)
    pts, wts = simplex_rule(3, 4)
    for K in (0, 5, 17, 40):
        J = Js[K]
        det = np.linalg.det(J)
        Phi = ref.eval(pts)
        if family in ("N1curl", "N2curl"):
            phys = np.einsum("ab,pjb->pja", np.linalg.inv(J).T, Phi)
        else:
            phys = np.einsum("ab,pjb->pja", J / det, Phi)
        Mq = abs(det) * np.einsum("p,pia,pja->ij", wts, phys, phys)
        assert np.max(np.abs(Mq - mats[K])) < 1e-13 * np.max(np.abs(mats[K]))


@pytest.mark.parametrize("d,k", [(2, 1), (2, 3), (2, 4), (3, 2), (3, 4)])
def test_bernstein_closed_form_mass(d, k):
    """int_T B_a B_b = (k!)^2 (a+b)! / (a! b! (2k+d)!) on the unit simplex
    (multi-index factorials are products over the d+1 entries)."""
    from math import factorial, prod
    e = fe.reference_element("B", d, k)
    alphas = []
    for edim in range(d + 1):
        for verts in fe.local_entities(d, edim):
            idxs = [(k,)] if edim == 0 else fe.interior_multi_indices(len(verts), k)
            for beta in idxs:
                a = [0] * (d + 1)
                for v, b in zip(verts, beta):
                    a[v] = b
                alphas.append(a)
    fac = lambda a: prod(factorial(x) for x in a)            # noqa: E731
    M = np.array([[factorial(k) ** 2 * fac([x + y for x, y in zip(a, b)]) / (fac(a) * fac(b) * factorial(2 * k + d))
                   for b in alphas] for a in alphas])
    assert np.max(np.abs(M - e.mass)) <= 1e-15 * np.max(M)


@pytest.mark.parametrize("d,k", [(2, 3), (3, 4)])
def test_bernstein_partition_of_unity_and_positivity(d, k):
    e = fe.reference_element("B", d, k)
    pts, _ = simplex_rule(d, 6)
    v = e.eval(pts)[:, :, 0]
    assert np.allclose(v.sum(axis=1), 1.0, atol=1e-14)
    assert v.min() >= -1e-15
    # vertex functions are 1 at their vertex and every other function vanishes there
    V = e.eval(np.array(fe.ref_vertices(d), dtype=float))[:, :, 0]
    assert np.allclose(V[:, :d + 1], np.eye(d + 1), atol=1e-15) and np.allclose(V[:, d + 1:], 0.0, atol=1e-15)


@pytest.mark.parametrize("d,k", [(2, 3), (3, 2), (3, 3)])
def test_bernstein_global_conformity_and_l2_norm(d, k):
    """The local Bernstein coefficients of one global polynomial agree on
    every shared entity (so P is 0/1 with the sorted-vertex numbering), and
    u' M u equals its L2 norm squared."""
    ref = fe.reference_element("B", d, k)
    coords, cells = mesh.structured_mesh(d, 2, jitter=0.2, seed=6)
    pr = assembly.Problem(ref, coords, cells, need_bras=False)
    c = np.array([0.4, -1.3, 0.8])[:d]
    f = lambda x: 1.0 + (x @ c) ** k - 0.5 * x[:, 0] * x[:, -1]      # noqa: E731
    Js = mesh.jacobians(coords, cells)
    pts, wts = simplex_rule(d, 2 * k + 2)
    B = ref.eval(pts)[:, :, 0]
    w = np.empty((len(cells), ref.n_loc))
    for K in range(len(cells)):
        x = coords[cells[K, 0]] + pts @ Js[K].T
        w[K] = np.linalg.lstsq(B, f(x), rcond=None)[0]               # exact: f is in the local space
    u = np.zeros(pr.n)
    u[pr.pi.ravel()] = w.ravel()
    assert np.max(np.abs(w - u[pr.pi])) < 1e-11
    tot = sum(abs(np.linalg.det(Js[K])) * np.sum(wts * f(coords[cells[K, 0]] + pts @ Js[K].T) ** 2)
              for K in range(len(cells)))
    assert abs(u @ (pr.M @ u) - tot) < 1e-11 * tot
