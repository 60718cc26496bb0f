"""Polynomials on reference simplices, with exact monomial integrals.

A polynomial in d variables is a dict {exponent tuple: coefficient}.
Coefficients may be Fractions (exact) or floats.  The reference d-simplex is
conv{0, e_1, ..., e_d}; on it

    integral of x^a = a_1! ... a_d! / (|a| + d)!

(the Dirichlet integral), which is exact in rational arithmetic.

Orthonormal polynomials on an entity are obtained by Gram-Schmidt of the
monomials in the fixed order `monomials(d, q)` (total degree ascending, then
exponent tuples in descending lexicographic order), in exact rational
arithmetic; normalisation (a square root) is the only inexact step.
"""
from fractions import Fraction
from functools import lru_cache
import itertools
import math

import numpy as np


def monomials(d, q):
    """Exponent tuples of total degree <= q, degree ascending, lex-descending."""
    out = []
    for deg in range(q + 1):
        block = [a for a in itertools.product(range(deg + 1), repeat=d) if sum(a) == deg]
        block.sort(reverse=True)
        out.extend(block)
    return out


def homogeneous(d, q):
    return [a for a in monomials(d, q) if sum(a) == q]


@lru_cache(maxsize=None)
def monomial_integral(a):
    """Exact integral of x^a over the reference |a|-dimensional simplex (Fraction)."""
    d = len(a)
    num = 1
    for ai in a:
        num *= math.factorial(ai)
    return Fraction(num, math.factorial(sum(a) + d))


def integrate(p, d):
    tot = 0
    for a, c in p.items():
        if len(a) != d:
            raise ValueError("dimension mismatch")
        tot = tot + c * monomial_integral(a)
    return tot


def mul(p, q):
    out = {}
    for a, ca in p.items():
        for b, cb in q.items():
            e = tuple(x + y for x, y in zip(a, b))
            out[e] = out.get(e, 0) + ca * cb
    return out


def add(p, q, s=1):
    out = dict(p)
    for a, c in q.items():
        out[a] = out.get(a, 0) + s * c
    return out


def scale(p, s):
    return {a: c * s for a, c in p.items()}


def const(d, c):
    return {(0,) * d: c}


def var(d, i):
    e = [0] * d
    e[i] = 1
    return {tuple(e): 1}


def power(p, k, d):
    out = const(d, 1)
    for _ in range(k):
        out = mul(out, p)
    return out


def compose_affine(p, v0, A):
    """Return p(v0 + A s) as a polynomial in s (A is d x d', v0 length d)."""
    d = len(v0)
    dp = len(A[0]) if d else 0
    lin = []
    for i in range(d):
        li = const(dp, v0[i])
        for j in range(dp):
            if A[i][j] != 0:
                li = add(li, scale(var(dp, j), A[i][j]))
        lin.append(li)
    out = {}
    cache = {}
    for a, c in p.items():
        term = const(dp, c)
        for i, ai in enumerate(a):
            if ai:
                key = (i, ai)
                if key not in cache:
                    cache[key] = power(lin[i], ai, dp)
                term = mul(term, cache[key])
        out = add(out, term)
    return out


def evaluate(p, x):
    tot = 0.0
    for a, c in p.items():
        v = float(c)
        for xi, ai in zip(x, a):
            v *= float(xi) ** ai
        tot += v
    return tot


def inner(p, q, d):
    return integrate(mul(p, q), d)


@lru_cache(maxsize=None)
def orthogonal_rational(d, q):
    """Exact orthogonal (unnormalised) polynomials on the reference d-simplex.

    Gram-Schmidt of monomials(d, q) with the L2 inner product of the
    reference simplex.  Returns a tuple of (poly dict with Fraction
    coefficients, squared norm Fraction).
    """
    basis = []
    for a in monomials(d, q):
        p = {a: Fraction(1)}
        for (b, nb) in basis:
            c = inner(p, b, d) / nb
            p = add(p, b, -c)
        p = {k: v for k, v in p.items() if v != 0}
        basis.append((p, inner(p, p, d)))
    return tuple(basis)


def orthonormal_float(d, q):
    """Orthonormal polynomials on the reference simplex (float coefficients)."""
    out = []
    for p, n2 in orthogonal_rational(d, q):
        s = 1.0 / math.sqrt(float(n2))
        out.append({a: float(c) * s for a, c in p.items()})
    return out


def to_dense(p, mons):
    """Coefficient vector of p over the monomial list mons (float)."""
    index = {a: i for i, a in enumerate(mons)}
    v = np.zeros(len(mons))
    for a, c in p.items():
        if c != 0:
            v[index[a]] += float(c)
    return v


def gram_matrix(d, mons):
    """G[i, j] = integral of x^(mons[i] + mons[j]) over the reference simplex."""
    m = len(mons)
    G = np.empty((m, m))
    for i in range(m):
        for j in range(i, m):
            e = tuple(x + y for x, y in zip(mons[i], mons[j]))
            G[i, j] = G[j, i] = float(monomial_integral(e))
    return G
