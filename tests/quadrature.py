"""Independent Gauss-Legendre / Duffy quadrature used by the oracle pins.

Deliberately a different route from the oracle's exact monomial integrals:
tensor Gauss-Legendre on [0,1]^d pushed to the reference simplex by the
collapsed (Duffy) map.
"""
import numpy as np


def gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return (x + 1.0) / 2.0, w / 2.0


def simplex_rule(d, n):
    """Points [npts, d] and weights on conv{0, e_1, .., e_d}, exact for degree
    <= 2n - 1 - (d - 1)."""
    x, w = gauss01(n)
    if d == 1:
        return x[:, None], w
    if d == 2:
        U, V = np.meshgrid(x, x, indexing="ij")
        WU, WV = np.meshgrid(w, w, indexing="ij")
        pts = np.stack([U, (1 - U) * V], axis=-1).reshape(-1, 2)
        wts = (WU * WV * (1 - U)).ravel()
        return pts, wts
    U, V, W = np.meshgrid(x, x, x, indexing="ij")
    WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
    pts = np.stack([U, (1 - U) * V, (1 - U) * (1 - V) * W], axis=-1).reshape(-1, 3)
    wts = (WU * WV * WW * (1 - U) ** 2 * (1 - V)).ravel()
    return pts, wts


def orthonormal_numeric(d, q, n=12):
    """Orthonormal basis of P_q on the reference d-simplex by modified
    Gram-Schmidt under this quadrature; returns a function mapping points
    [npts, d] to values [npts, dim P_q]."""
    from itertools import product
    exps = []
    for deg in range(q + 1):
        blk = [a for a in product(range(deg + 1), repeat=d) if sum(a) == deg]
        blk.sort(reverse=True)
        exps.extend(blk)
    pts, wts = simplex_rule(d, n)
    V = np.stack([np.prod(pts ** np.array(a), axis=1) for a in exps], axis=1)
    R = np.zeros((len(exps), len(exps)))
    Q = V.copy()
    for j in range(len(exps)):
        for i in range(j):
            c = np.sum(wts * Q[:, i] * Q[:, j])
            Q[:, j] -= c * Q[:, i]
            R[i, j] += c
        nrm = np.sqrt(np.sum(wts * Q[:, j] ** 2))
        Q[:, j] /= nrm
        R[j, j] = nrm
    Rinv = np.linalg.inv(R)

    def ev(x):
        x = np.atleast_2d(x)
        Vx = np.stack([np.prod(x ** np.array(a), axis=1) for a in exps], axis=1)
        return Vx @ Rinv
    return ev


def _exps(d, q, homogeneous=False):
    from itertools import product
    out = []
    for deg in range(q if homogeneous else 0, q + 1):
        blk = [a for a in product(range(deg + 1), repeat=d) if sum(a) == deg]
        blk.sort(reverse=True)
        out.extend(blk)
    return out


def moment_fields_numeric(kind, m, j, n=12):
    """RT_j (kind "RT") or N1curl_j test fields on the m-simplex, in the fixed
    spanning order of the second-kind moments ([P_{j-1}]^m component-major,
    then x q, (-y q, x q) or x cross (e_c q) with dependent ones skipped),
    orthonormalised in that order under this quadrature.  Returns a function
    mapping points [npts, m] to values [npts, nfields, m]."""
    if j < 1:
        return None
    mono = lambda x, a: np.prod(x ** np.array(a), axis=1)       # noqa: E731
    fields = []                                                 # callables x -> [npts, m]
    for c in range(m):
        for a in _exps(m, j - 1):
            fields.append(lambda x, c=c, a=a: np.eye(m)[c][None, :] * mono(x, a)[:, None])
    for a in _exps(m, j - 1, homogeneous=True):
        if kind == "RT":
            fields.append(lambda x, a=a: x * mono(x, a)[:, None])
        elif m == 2:
            fields.append(lambda x, a=a: np.stack([-x[:, 1], x[:, 0]], axis=1) * mono(x, a)[:, None])
        else:
            for c in range(3):
                fields.append(lambda x, a=a, c=c: np.cross(x, np.eye(3)[c][None, :]) * mono(x, a)[:, None])
    pts, wts = simplex_rule(m, n)
    vals = [f(pts) for f in fields]
    # skip dependent fields (greedy, in order), then Gram-Schmidt in order
    kept, Q, R_rows = [], [], []
    for i, v in enumerate(vals):
        w = v.copy()
        coef = np.zeros(len(vals))
        coef[i] = 1.0
        for qv, qc in zip(Q, R_rows):
            c = np.sum(wts[:, None] * qv * w)
            w = w - c * qv
            coef = coef - c * qc
        nrm = np.sqrt(np.sum(wts[:, None] * w * w))
        if nrm < 1e-9 * np.sqrt(np.sum(wts[:, None] * v * v)):
            continue
        kept.append(i)
        Q.append(w / nrm)
        R_rows.append(coef / nrm)
    C = np.array(R_rows)                                        # orthonormal = C @ fields

    def ev(x):
        x = np.atleast_2d(x)
        F = np.stack([f(x) for f in fields], axis=1)            # [npts, nall, m]
        return np.einsum("qa,pam->pqm", C, F)
    return ev
