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
