"""Closed forms for diagonal (Fermat) hypersurfaces (test infrastructure only).

Weil's Gauss-sum formula: for X: x_0^d + ... + x_n^d = 0 over F_p with
d | p - 1, the eigenvalues of Frobenius on primitive middle cohomology are
    alpha_e = (-1)^(n+1) g(chi^e_0) ... g(chi^e_n) / p
over e in [1, d-1]^(n+1) with sum e = 0 mod d, chi a character of order d and
g the Gauss sum; so Q(T) = prod_e (1 - alpha_e T).  Counting points of the
affine cone with additive characters gives this directly, and Hasse-Davenport
lifts it to every F_{p^k}.  For d | p + 1 a Fermat CURVE is supersingular and
maximal over F_{p^2}: Q(T) = (1 + p T^2)^g.
"""
import itertools
from math import comb

import mpmath


def primitive_root(p):
    for g in range(2, p):
        if all(pow(g, (p - 1) // f, p) != 1 for f in _prime_factors(p - 1)):
            return g
    raise ValueError


def _prime_factors(x):
    out, k = set(), 2
    while k * k <= x:
        while x % k == 0:
            out.add(k)
            x //= k
        k += 1
    if x > 1:
        out.add(x)
    return out


def gauss_sum(p, d, e, g0):
    """g(chi^e) = sum_{x != 0} chi^e(x) exp(2 pi i x / p), chi(g0^t) = exp(2 pi i t / d),
    in mpmath complex arithmetic at the working precision."""
    tot = mpmath.mpc(0)
    xt = 1
    for t in range(p - 1):
        tot += mpmath.expjpi(mpmath.mpf(2 * (e * t % d)) / d) * mpmath.expjpi(mpmath.mpf(2 * xt) / p)
        xt = xt * g0 % p
    return tot


def fermat_lpoly(nv, d, p, dps=120):
    """Exact integer Q(T) of the Fermat hypersurface of degree d in P^(nv-1).

    d | p-1: prod_e (1 - alpha_e T) expanded in mpmath at ``dps`` digits and
    rounded (the coefficients are rational integers far below 10^dps).
    Curves with d | p+1: (1 + p T^2)^g."""
    n = nv - 1
    if (p - 1) % d == 0:
        with mpmath.workdps(dps):
            g0 = primitive_root(p)
            gs = {e: gauss_sum(p, d, e, g0) for e in range(1, d)}
            poly = [mpmath.mpc(1)]
            for es in itertools.product(range(1, d), repeat=nv):
                if sum(es) % d:
                    continue
                alpha = mpmath.mpc((-1) ** (n + 1)) / p
                for e in es:
                    alpha *= gs[e]
                nxt = poly + [mpmath.mpc(0)]
                for i in range(len(poly)):
                    nxt[i + 1] -= alpha * poly[i]
                poly = nxt
            out = []
            for c in poly:
                k = int(mpmath.nint(c.real))
                assert abs(c.real - k) < mpmath.mpf(10) ** (-20) and abs(c.imag) < mpmath.mpf(10) ** (-20)
                out.append(k)
            return out
    if n == 2 and (p + 1) % d == 0:
        g = (d - 1) * (d - 2) // 2
        out = [0] * (2 * g + 1)
        for k in range(g + 1):
            out[2 * k] = comb(g, k) * p ** k
        return out
    raise ValueError("no closed form implemented for this (d, p)")


def fermat_coeffs(nv, d):
    """Coefficient list (lex-descending monomial order) of x_0^d + ... + x_n^d."""
    from .poly import monomials
    mons = monomials(nv, d)
    return [1 if max(m) == d else 0 for m in mons]
