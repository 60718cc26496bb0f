"""Reference finite elements and reference mass matrices (oracle side).

Families (Section 3 names them after Firedrake; the readings used here):

* "P"      H1 Lagrange P_p, nodal basis at the "spectral" (GLL-based) nodes
           of the recursive construction of Isaac (SIAM J. Sci. Comput. 2020):
           on an edge the nodes are the p+1 Gauss-Lobatto-Legendre points; a
           point with barycentric multi-index alpha (all entries >= 1, sum n)
           inside a k-simplex, k >= 2, is the average of the points of the
           facet multi-indices alpha without entry i (sum n - alpha_i),
           weighted by n - alpha_i.  A multi-index with zero entries lives on
           the sub-simplex of its non-zero entries.
* "N1curl" first-kind Nedelec N1curl_k = [P_{k-1}]^d + S_k with S_k the
           degree-k homogeneous fields u with x . u = 0 (3D) or (-y, x) P~_{k-1}
           (2D).  Degrees of freedom are integral moments.
* "RT"     Raviart-Thomas RT_k = [P_{k-1}]^d + x P~_{k-1}, integral moments.
* "N2curl" second-kind Nedelec, the full space [P_k]^d (covariant Piola).
* "BDM"    Brezzi-Douglas-Marini, the full space [P_k]^d (contravariant Piola).
* "B"      H1 P_p in the Bernstein basis (Section 3, Table h1_mass_solve):
           B_alpha = p!/(alpha_0! ... alpha_d!) lambda_0^alpha_0 ... lambda_d^alpha_d
           over barycentric multi-indices |alpha| = p, lambda_0 = 1 - sum x_i,
           lambda_i = x_i.  A function whose multi-index vanishes off a
           sub-simplex is supported on it there, so with cells listing sorted
           vertices neighbouring cells agree on shared functions; local order
           as for Lagrange nodes (same multi-indices).

Moment degrees of freedom (the variant is not stated in the paper; this is
the integral-moment reading).  Entities are taken with sorted vertices
(a < b < c), parametrised by x(s) = v_a + s (v_b - v_a) (+ t (v_c - v_a)):
  N1curl edge   int_0^1 (u . t) q ds,  t = v_b - v_a,      q in P_{k-1}
  N1curl face   int_f (u . t_1) q, then int_f (u . t_2) q,
                t_1 = v_b - v_a, t_2 = v_c - v_a,           q in P_{k-2}
  RT face (3D)  int_f (u . n) q,  n = t_1 x t_2,            q in P_{k-1}
  RT edge (2D)  int_0^1 (u . n) q ds, n = (t_y, -t_x),      q in P_{k-1}
  interior      int_K u_c q, component-major,   q in P_{k-2} (RT, 2D N1curl)
                                                or P_{k-3} (3D N1curl)
with q running over the orthonormal polynomials of the entity in parameter
coordinates (oracle.poly).  Second-kind families (classical moments; the
test spaces are listed in the design notes):
  N2curl edge   int_0^1 (u . t) q ds,                       q in P_k
  N2curl face   int_f (u . t_1) q_1 + (u . t_2) q_2,        (q_1, q_2) in RT_{k-1}
                                                            (face parameters)
  N2curl int.   int_K u . q,  q in RT_{k-1} (2D) or RT_{k-2} (3D)
  BDM facet     int (u . n) q,  n as for RT,                q in P_k
  BDM interior  int_K u . q,  q in N1curl_{k-1}
where the RT_j / N1curl_j test fields are the monomial spanning fields
[P_{j-1}]^m (component-major), then x q (RT), (-y, x) q (2D N1curl) or
x cross (e_c q) (3D N1curl; q outer, c inner, each kept only if independent
of the fields kept before it), q over the homogeneous monomials of degree
j - 1, and then orthonormalised in that order (Gram-Schmidt under the L2
inner product of the entity's parameter domain, i.e. f L^-T with L the
Cholesky factor of their Gram matrix).  With these functionals a field's degrees of
freedom are unchanged by the covariant / contravariant Piola maps, so shared
degrees of freedom agree between neighbouring cells and P stays 0/1.

Local degree-of-freedom order: vertices, edges (local vertex pairs in lex
order), faces (3D; local triples in lex order), interior.  Lagrange nodes
inside an entity are ordered by their barycentric multi-index over the
entity's vertices, in descending lexicographic order.

Reference mass matrices (eq. piola_mass_pullbacks): for H1
Mhat_ij = int phi_i phi_j; for vector families Mhat^{ab}_ij = int phi_i^a
phi_j^b, so that the physical element matrix is sum_ab G_ab Mhat^{ab}.

Arithmetic: the space bases, functionals and monomial integrals are exact
rationals; the nodal basis (inverse of the functional Vandermonde) and the
mass tables are computed in 34-digit mpmath and rounded to float64 once at
the end, so the tables are correct to about one unit in the last place
despite the monomial representation's conditioning.
"""
from dataclasses import dataclass, field
from fractions import Fraction
from functools import lru_cache
import itertools
import math

import mpmath as mp
import numpy as np

from . import poly

DPS = 34


def _mpf(x):
    if isinstance(x, Fraction):
        return mp.mpf(x.numerator) / x.denominator
    return mp.mpf(x)


# ----------------------------------------------------------------------------
# GLL points and recursive nodes
# ----------------------------------------------------------------------------

def _legendre_and_derivative(n, x):
    """P_n(x) and P_n'(x) on [-1, 1] by the three-term recurrence."""
    p0, p1 = mp.mpf(1), x
    if n == 0:
        return p0, mp.mpf(0)
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    dp = n * (x * p1 - p0) / (x * x - 1)
    return p1, dp


def gll01_mp(n):
    """The n+1 Gauss-Lobatto-Legendre points on [0, 1] (ascending), mpmath."""
    with mp.workdps(DPS):
        if n < 1:
            raise ValueError("n >= 1")
        if n == 1:
            return [mp.mpf(0), mp.mpf(1)]
        if n == 2:
            return [mp.mpf(0), mp.mpf(1) / 2, mp.mpf(1)]
        if n == 3:
            r = 1 / mp.sqrt(5)
            return [mp.mpf(0), (1 - r) / 2, (1 + r) / 2, mp.mpf(1)]
        if n == 4:
            r = mp.sqrt(21) / 14
            return [mp.mpf(0), mp.mpf(1) / 2 - r, mp.mpf(1) / 2, mp.mpf(1) / 2 + r, mp.mpf(1)]
        guess = np.sort(np.polynomial.legendre.Legendre.basis(n).deriv().roots().real)
        pts = [mp.mpf(0)]
        for g in guess:
            # interior GLL points are the roots of P_n'; Newton on P_n' with
            # P_n'' = (2x P_n' - n(n+1) P_n) / (1 - x^2)
            x = mp.mpf(float(g))
            for _ in range(60):
                pn, dpn = _legendre_and_derivative(n, x)
                d2 = (2 * x * dpn - n * (n + 1) * pn) / (1 - x * x)
                step = dpn / d2
                x -= step
                if abs(step) < mp.mpf(10) ** (-DPS + 2):
                    break
            pts.append((x + 1) / 2)
        pts.append(mp.mpf(1))
        return pts


def gll01(n):
    """The n+1 Gauss-Lobatto-Legendre points on [0, 1], ascending (float64)."""
    return np.array([float(x) for x in gll01_mp(n)])


def recursive_bary(alpha):
    """Barycentric coordinates of the recursive GLL node with multi-index alpha (mpmath)."""
    alpha = tuple(int(a) for a in alpha)
    support = [i for i, a in enumerate(alpha) if a > 0]
    sub = _rec_full(tuple(alpha[i] for i in support))
    out = [mp.mpf(0)] * len(alpha)
    for i, v in zip(support, sub):
        out[i] = v
    return out


@lru_cache(maxsize=None)
def _rec_full(alpha):
    with mp.workdps(DPS):
        n = sum(alpha)
        k = len(alpha)
        if k == 1:
            return (mp.mpf(1),)
        if k == 2:
            g = gll01_mp(n)[alpha[1]]
            return (1 - g, g)
        acc = [mp.mpf(0)] * k
        wsum = 0
        for i in range(k):
            w = n - alpha[i]
            facet = _rec_full(alpha[:i] + alpha[i + 1:])
            b = list(facet[:i]) + [mp.mpf(0)] + list(facet[i:])
            acc = [a + w * bb for a, bb in zip(acc, b)]
            wsum += w
        return tuple(a / wsum for a in acc)


def interior_multi_indices(k, n):
    """Multi-indices of length k, all entries >= 1, sum n, descending lex order."""
    out = [a for a in itertools.product(range(1, n + 1), repeat=k) if sum(a) == n]
    out.sort(reverse=True)
    return out


# ----------------------------------------------------------------------------
# Reference simplex and its sub-entities
# ----------------------------------------------------------------------------

def ref_vertices(d):
    return [tuple(0 for _ in range(d))] + [tuple(1 if j == i else 0 for j in range(d)) for i in range(d)]


def local_entities(d, edim):
    return list(itertools.combinations(range(d + 1), edim + 1))


@dataclass
class RefElement:
    family: str
    dim: int
    degree: int
    ncomp: int
    n_loc: int
    dofs_per_entity: tuple          # DOFs per vertex, edge, (face,) cell
    mons: list
    basis: np.ndarray               # [n_loc, ncomp, m] monomial coefficients (float64)
    mass: np.ndarray                # H1: [n_loc, n_loc]; vector: [d, d, n_loc, n_loc]
    nodes: np.ndarray = field(default=None)   # Lagrange nodes [n_loc, d]

    def eval(self, x):
        """Basis values at points x [npts, d] -> [npts, n_loc, ncomp] (float64)."""
        x = np.atleast_2d(np.asarray(x, dtype=float))
        V = np.stack([np.prod(x ** np.array(a), axis=1) for a in self.mons], axis=1)
        return np.einsum("pm,jcm->pjc", V, self.basis)


def _entity_param(d, verts):
    """v0 and tangent matrix A (d x k) of the entity with local vertices verts."""
    rv = ref_vertices(d)
    v0 = [Fraction(c) for c in rv[verts[0]]]
    A = [[Fraction(rv[verts[j]][i] - rv[verts[0]][i]) for j in range(1, len(verts))] for i in range(d)]
    return v0, A


def _moment_row(d, mons, verts, direction, q_rational, q_norm2):
    """ell[c][mu] = int_entity (e_c x^mu . direction) q  (q = orthonormal polynomial)."""
    v0, A = _entity_param(d, verts)
    k = len(verts) - 1
    s = 1 / mp.sqrt(_mpf(q_norm2))
    ell = [[mp.mpf(0)] * len(mons) for _ in range(d)]
    for mi, mu in enumerate(mons):
        restricted = poly.compose_affine({mu: Fraction(1)}, v0, A)
        val = poly.integrate(poly.mul(restricted, q_rational), k)
        for c in range(d):
            if direction[c] != 0:
                ell[c][mi] = _mpf(val * direction[c]) * s
    return ell


def _interior_row(d, mons, comp, q_rational, q_norm2):
    s = 1 / mp.sqrt(_mpf(q_norm2))
    ell = [[mp.mpf(0)] * len(mons) for _ in range(d)]
    for mi, mu in enumerate(mons):
        ell[comp][mi] = _mpf(poly.integrate(poly.mul({mu: Fraction(1)}, q_rational), d)) * s
    return ell


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def rational_null_space(A):
    """Exact basis of ker A for a matrix of integers / Fractions (Gauss-Jordan)."""
    rows = [[Fraction(v) for v in r] for r in A]
    nr, nc = len(rows), len(rows[0])
    pivots = []
    r = 0
    for c in range(nc):
        piv = next((i for i in range(r, nr) if rows[i][c] != 0), None)
        if piv is None:
            continue
        rows[r], rows[piv] = rows[piv], rows[r]
        pv = rows[r][c]
        rows[r] = [v / pv for v in rows[r]]
        for i in range(nr):
            if i != r and rows[i][c] != 0:
                f = rows[i][c]
                rows[i] = [a - f * b for a, b in zip(rows[i], rows[r])]
        pivots.append(c)
        r += 1
        if r == nr:
            break
    free = [c for c in range(nc) if c not in pivots]
    basis = []
    for f in free:
        v = [Fraction(0)] * nc
        v[f] = Fraction(1)
        for i, pc in enumerate(pivots):
            v[pc] = -rows[i][f]
        basis.append(v)
    return basis


def _space_basis(family, d, k, mons):
    """A basis of the element's polynomial space: list of sparse fields
    {(component, monomial index): Fraction}."""
    index = {a: i for i, a in enumerate(mons)}
    if family == "P":
        return [{(0, i): Fraction(1)} for i in range(len(mons))]
    if family in ("N2curl", "BDM"):
        return [{(c, i): Fraction(1)} for c in range(d) for i in range(len(mons))]
    vecs = []
    for c in range(d):
        for mu in poly.monomials(d, k - 1):
            vecs.append({(c, index[mu]): Fraction(1)})
    hom = poly.homogeneous(d, k - 1)
    if family == "RT":
        for mu in hom:
            v = {}
            for c in range(d):
                e = list(mu)
                e[c] += 1
                v[(c, index[tuple(e)])] = Fraction(1)
            vecs.append(v)
    elif family == "N1curl" and d == 2:
        for mu in hom:
            e0 = list(mu); e0[1] += 1
            e1 = list(mu); e1[0] += 1
            vecs.append({(0, index[tuple(e0)]): Fraction(-1), (1, index[tuple(e1)]): Fraction(1)})
    elif family == "N1curl" and d == 3:
        # kernel of u -> x . u on degree-k homogeneous fields
        homk = poly.homogeneous(3, k)
        homk1 = poly.homogeneous(3, k + 1)
        idx1 = {a: i for i, a in enumerate(homk1)}
        A = [[0] * (3 * len(homk)) for _ in homk1]
        for c in range(3):
            for j, mu in enumerate(homk):
                e = list(mu)
                e[c] += 1
                A[idx1[tuple(e)]][c * len(homk) + j] = 1
        for col in rational_null_space(A):
            v = {}
            for c in range(3):
                for j, mu in enumerate(homk):
                    if col[c * len(homk) + j] != 0:
                        v[(c, index[mu])] = col[c * len(homk) + j]
            vecs.append(v)
    else:
        raise ValueError(family)
    return vecs


def _functionals(family, d, k, mons):
    """Rows ell_i[c][mu] (mpmath) of the degree-of-freedom functionals, local order."""
    rows = []
    counts = [0] * (d + 1)
    rv = ref_vertices(d)
    if family == "P":
        nodes = []
        for edim in range(d + 1):
            for verts in local_entities(d, edim):
                idxs = [(k,)] if edim == 0 else interior_multi_indices(len(verts), k)
                counts[edim] = len(idxs)
                for beta in idxs:
                    alpha = [0] * (d + 1)
                    for v, b in zip(verts, beta):
                        alpha[v] = b
                    bary = recursive_bary(alpha)
                    x = [sum(bary[v] * rv[v][i] for v in range(d + 1)) for i in range(d)]
                    nodes.append(x)
                    row = []
                    for a in mons:
                        t = mp.mpf(1)
                        for xi, ai in zip(x, a):
                            t *= xi ** ai
                        row.append(t)
                    rows.append([row])
        return rows, tuple(counts), np.array([[float(c) for c in x] for x in nodes])

    if family in ("N2curl", "BDM"):
        return _second_kind_functionals(family, d, k, mons)

    if family == "N1curl" or (family == "RT" and d == 2):
        qs = poly.orthogonal_rational(1, k - 1)
        for verts in local_entities(d, 1):
            t = tuple(rv[verts[1]][i] - rv[verts[0]][i] for i in range(d))
            direction = t if family == "N1curl" else (t[1], -t[0])
            for q, n2 in qs:
                rows.append(_moment_row(d, mons, verts, direction, q, n2))
        counts[1] = len(qs)
    if d == 3:
        for verts in local_entities(3, 2):
            t1 = tuple(rv[verts[1]][i] - rv[verts[0]][i] for i in range(3))
            t2 = tuple(rv[verts[2]][i] - rv[verts[0]][i] for i in range(3))
            if family == "RT":
                qs = poly.orthogonal_rational(2, k - 1)
                nrm = _cross(t1, t2)
                for q, n2 in qs:
                    rows.append(_moment_row(3, mons, verts, nrm, q, n2))
                counts[2] = len(qs)
            else:
                qs = poly.orthogonal_rational(2, k - 2) if k >= 2 else ()
                for tt in (t1, t2):
                    for q, n2 in qs:
                        rows.append(_moment_row(3, mons, verts, tt, q, n2))
                counts[2] = 2 * len(qs)
    qdeg = k - 2 if (family == "RT" or d == 2) else k - 3
    nint = 0
    if qdeg >= 0:
        qs = poly.orthogonal_rational(d, qdeg)
        for c in range(d):
            for q, n2 in qs:
                rows.append(_interior_row(d, mons, c, q, n2))
        nint = d * len(qs)
    counts[d] = nint
    return rows, tuple(counts), None


def _is_independent(kept, v):
    """Whether the rational vector v is independent of the rows in kept."""
    rows = [list(r) for r in kept] + [list(v)]
    return len(rational_null_space(list(map(list, zip(*rows))))) == 0


def test_fields(kind, m, j):
    """Monomial spanning fields of RT_j or N1curl_j on the m-simplex, in the
    fixed order stated in the module docstring.  A field is a list of m
    polynomials (dicts exponent -> Fraction)."""
    if j < 1:
        return []
    out = []
    for c in range(m):
        for mu in poly.monomials(m, j - 1):
            f = [{} for _ in range(m)]
            f[c] = {mu: Fraction(1)}
            out.append(f)
    hom = poly.homogeneous(m, j - 1)
    if kind == "RT":
        for mu in hom:
            f = []
            for c in range(m):
                e = list(mu)
                e[c] += 1
                f.append({tuple(e): Fraction(1)})
            out.append(f)
    elif m == 2:
        for mu in hom:
            e0 = list(mu); e0[1] += 1
            e1 = list(mu); e1[0] += 1
            out.append([{tuple(e0): Fraction(-1)}, {tuple(e1): Fraction(1)}])
    else:
        # x cross (e_c q): component c+1 gets x_{c+2} q, component c+2 gets -x_{c+1} q
        homj = poly.homogeneous(3, j)
        col = {a: i for i, a in enumerate(homj)}
        kept = []
        for mu in hom:
            for c in range(3):
                i1, i2 = (c + 1) % 3, (c + 2) % 3
                ea = list(mu); ea[i2] += 1
                eb = list(mu); eb[i1] += 1
                f = [{} for _ in range(3)]
                f[i1] = {tuple(ea): Fraction(1)}
                f[i2] = {tuple(eb): Fraction(-1)}
                v = [Fraction(0)] * (3 * len(homj))
                v[i1 * len(homj) + col[tuple(ea)]] = Fraction(1)
                v[i2 * len(homj) + col[tuple(eb)]] = Fraction(-1)
                if _is_independent(kept, v):
                    kept.append(v)
                    out.append(f)
    return out


def _field_moment_row(d, mons, verts, dirs, field):
    """ell[c][mu] = int_entity sum_i (e_c x^mu . dirs_i) field_i  over the
    entity's parameter domain (dirs_i: the i-th parameter tangent, or a unit
    direction)."""
    v0, A = _entity_param(d, verts)
    k = len(verts) - 1
    ell = [[mp.mpf(0)] * len(mons) for _ in range(d)]
    for mi, mu in enumerate(mons):
        restricted = poly.compose_affine({mu: Fraction(1)}, v0, A)
        for dv, q in zip(dirs, field):
            if not q:
                continue
            val = poly.integrate(poly.mul(restricted, q), k)
            for c in range(d):
                if dv[c] != 0:
                    ell[c][mi] += _mpf(val * dv[c])
    return ell


def _orthonormal_rows(raw, fields, m):
    """Rows of the Gram-Schmidt-orthonormalised test fields: sum_j Linv[i, j] raw_j,
    G = L L^T the Gram matrix of the fields on the m-simplex."""
    nf = len(fields)
    if nf == 0:
        return []
    G = mp.matrix(nf, nf)
    for i in range(nf):
        for j in range(nf):
            tot = Fraction(0)
            for a, b in zip(fields[i], fields[j]):
                if a and b:
                    tot += poly.integrate(poly.mul(a, b), m)
            G[i, j] = _mpf(tot)
    Linv = mp.inverse(mp.cholesky(G))
    out = []
    for i in range(nf):
        row = [[mp.mpf(0)] * len(raw[0][0]) for _ in range(len(raw[0]))]
        for j in range(i + 1):
            for c in range(len(row)):
                for mu in range(len(row[c])):
                    row[c][mu] += Linv[i, j] * raw[j][c][mu]
        out.append(row)
    return out


def _second_kind_functionals(family, d, k, mons):
    rows = []
    counts = [0] * (d + 1)
    rv = ref_vertices(d)
    if d == 2 or family == "N2curl":
        qs = poly.orthogonal_rational(1, k)
        for verts in local_entities(d, 1):
            t = tuple(rv[verts[1]][i] - rv[verts[0]][i] for i in range(d))
            direction = t if family == "N2curl" else (t[1], -t[0])
            for q, n2 in qs:
                rows.append(_moment_row(d, mons, verts, direction, q, n2))
        counts[1] = len(qs)
    if d == 3:
        for verts in local_entities(3, 2):
            t1 = tuple(rv[verts[1]][i] - rv[verts[0]][i] for i in range(3))
            t2 = tuple(rv[verts[2]][i] - rv[verts[0]][i] for i in range(3))
            if family == "BDM":
                qs = poly.orthogonal_rational(2, k)
                nrm = _cross(t1, t2)
                for q, n2 in qs:
                    rows.append(_moment_row(3, mons, verts, nrm, q, n2))
                counts[2] = len(qs)
            else:
                fs = test_fields("RT", 2, k - 1)
                raw = [_field_moment_row(3, mons, verts, (t1, t2), f) for f in fs]
                rows.extend(_orthonormal_rows(raw, fs, 2))
                counts[2] = len(fs)
    if family == "BDM":
        fs = test_fields("N1curl", d, k - 1)
    else:
        fs = test_fields("RT", d, k - 1 if d == 2 else k - 2)
    unit = [tuple(1 if i == c else 0 for i in range(d)) for c in range(d)]
    raw = [_field_moment_row(d, mons, tuple(range(d + 1)), unit, f) for f in fs]
    rows.extend(_orthonormal_rows(raw, fs, d))
    counts[d] = len(fs)
    return rows, tuple(counts), None


def _bernstein(d, k, mons):
    """Bernstein basis (exact rationals) in the local order of the Lagrange
    nodes: vertices, then edges, faces, interior, each entity's multi-indices
    in descending lexicographic order.  Returns (polynomials, counts)."""
    lam = [poly.add(poly.const(d, Fraction(1)), sum_vars(d), -1)] + [poly.var(d, i) for i in range(d)]
    out = []
    counts = [0] * (d + 1)
    for edim in range(d + 1):
        for verts in local_entities(d, edim):
            idxs = [(k,)] if edim == 0 else interior_multi_indices(len(verts), k)
            counts[edim] = len(idxs)
            for beta in idxs:
                alpha = [0] * (d + 1)
                for v, b in zip(verts, beta):
                    alpha[v] = b
                coef = Fraction(math.factorial(k), math.prod(math.factorial(a) for a in alpha))
                p = poly.const(d, coef)
                for i, a in enumerate(alpha):
                    p = poly.mul(p, poly.power(lam[i], a, d))
                out.append(p)
    return out, tuple(counts)


def sum_vars(d):
    p = {}
    for i in range(d):
        p = poly.add(p, poly.var(d, i))
    return p


def _bernstein_element(dim, degree):
    mons = poly.monomials(dim, degree)
    index = {m: i for i, m in enumerate(mons)}
    polys, counts = _bernstein(dim, degree, mons)
    nb = len(polys)
    coef = [[Fraction(0)] * len(mons) for _ in range(nb)]
    for j, p in enumerate(polys):
        for e, c in p.items():
            coef[j][index[e]] += c
    mass = np.empty((nb, nb))
    for i in range(nb):
        for j in range(i, nb):
            v = poly.integrate(poly.mul(polys[i], polys[j]), dim)   # exact rational
            mass[i, j] = mass[j, i] = float(v)
    basis = np.array([[[float(c) for c in coef[j]]] for j in range(nb)])
    return RefElement("B", dim, degree, 1, nb, counts, mons, basis, mass, None)


@lru_cache(maxsize=None)
def reference_element(family, dim, degree):
    """Construct the reference element (basis coefficients and mass tables)."""
    if family not in ("P", "N1curl", "RT", "B", "N2curl", "BDM"):
        raise ValueError(family)
    if dim not in (2, 3) or degree < 1:
        raise ValueError("unsupported element")
    if family == "B":
        return _bernstein_element(dim, degree)
    with mp.workdps(DPS):
        mons = poly.monomials(dim, degree)
        m = len(mons)
        Psi = _space_basis(family, dim, degree, mons)
        rows, counts, nodes = _functionals(family, dim, degree, mons)
        nb = len(Psi)
        if len(rows) != nb:
            raise AssertionError("dof count %d != space dim %d" % (len(rows), nb))
        ncomp = 1 if family == "P" else dim
        # V[i, s] = L_i(psi_s)
        V = mp.matrix(nb, nb)
        for s_, psi in enumerate(Psi):
            for (c, mu), val in psi.items():
                fv = _mpf(val)
                for i in range(nb):
                    V[i, s_] += rows[i][c][mu] * fv
        C = mp.inverse(V)                    # phi_j = sum_s C[s, j] psi_s
        Phi = [[[mp.mpf(0)] * m for _ in range(ncomp)] for _ in range(nb)]
        for s_, psi in enumerate(Psi):
            for (c, mu), val in psi.items():
                fv = _mpf(val)
                for j in range(nb):
                    if C[s_, j] != 0:
                        Phi[j][c][mu] += C[s_, j] * fv
        G = mp.matrix(m, m)
        for i in range(m):
            for j in range(m):
                G[i, j] = _mpf(poly.monomial_integral(tuple(x + y for x, y in zip(mons[i], mons[j]))))
        comp = [mp.matrix([[Phi[j][c][mu] for mu in range(m)] for j in range(nb)]) for c in range(ncomp)]
        basis = np.array([[[float(Phi[j][c][mu]) for mu in range(m)] for c in range(ncomp)] for j in range(nb)])
        if ncomp == 1:
            Mm = comp[0] * G * comp[0].T
            mass = np.array([[float(Mm[i, j]) for j in range(nb)] for i in range(nb)])
            mass = 0.5 * (mass + mass.T)
        else:
            mass = np.empty((dim, dim, nb, nb))
            GT = [G * comp[b].T for b in range(dim)]
            for a in range(dim):
                for b in range(a, dim):
                    Mm = comp[a] * GT[b]
                    blk = np.array([[float(Mm[i, j]) for j in range(nb)] for i in range(nb)])
                    mass[a, b] = blk
                    mass[b, a] = blk.T
            for a in range(dim):
                mass[a, a] = 0.5 * (mass[a, a] + mass[a, a].T)
    return RefElement(family, dim, degree, ncomp, nb, counts, mons, basis, mass, nodes)


def element_dim(family, d, k):
    if family in ("P", "B"):
        return math.comb(k + d, d)
    if family == "RT":
        return d * math.comb(k - 1 + d, d) + math.comb(k - 1 + d - 1, d - 1)
    if family == "N1curl":
        return k * (k + 2) * (k + 3) // 2 if d == 3 else k * (k + 2)
    if family in ("N2curl", "BDM"):
        return d * math.comb(k + d, d)
    raise ValueError(family)
