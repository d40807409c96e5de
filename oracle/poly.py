"""Monomials and exact-integer polynomials (oracle; test infrastructure only).

Conventions (Section 2.1 notation): Homog_k is the space of homogeneous
polynomials of degree k in x_0..x_n; Homog_k = {0} for k < 0 and Homog_0 = {1}.
Monomials of a degree are listed in lexicographically DESCENDING order of
their exponent vectors (x_0^k first), which is also the coefficient order of
the library's input.
"""
from math import comb


def monomials(nv, deg):
    """All exponent tuples of length nv summing to deg, lex-descending."""
    if deg < 0:
        return []
    if nv == 1:
        return [(deg,)]
    out = []
    for e0 in range(deg, -1, -1):
        for rest in monomials(nv - 1, deg - e0):
            out.append((e0,) + rest)
    return out


def n_monomials(nv, deg):
    return comb(deg + nv - 1, nv - 1) if deg >= 0 else 0


def index_of(mons):
    return {m: i for i, m in enumerate(mons)}


def padd(a, b, q=None):
    out = dict(a)
    for e, c in b.items():
        out[e] = out.get(e, 0) + c
    if q is not None:
        out = {e: c % q for e, c in out.items()}
    return {e: c for e, c in out.items() if c != 0}


def pmul(a, b, q=None):
    out = {}
    for ea, ca in a.items():
        for eb, cb in b.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0) + ca * cb
    if q is not None:
        out = {e: c % q for e, c in out.items()}
    return {e: c for e, c in out.items() if c != 0}


def ppow(a, k, nv):
    out = {(0,) * nv: 1}
    for _ in range(k):
        out = pmul(out, a)
    return out


def pderiv(a, i):
    """Partial derivative d/dx_i."""
    out = {}
    for e, c in a.items():
        if e[i] > 0:
            e2 = list(e)
            e2[i] -= 1
            out[tuple(e2)] = out.get(tuple(e2), 0) + c * e[i]
    return {e: c for e, c in out.items() if c != 0}


def from_coeffs(nv, d, coeffs):
    """Polynomial from coefficients listed in lex-descending monomial order."""
    mons = monomials(nv, d)
    assert len(coeffs) == len(mons)
    return {m: int(c) for m, c in zip(mons, coeffs) if int(c) != 0}


def to_vector(poly, mons_index, q=None):
    v = [0] * len(mons_index)
    for e, c in poly.items():
        v[mons_index[e]] += c
    if q is not None:
        v = [x % q for x in v]
    return v
