"""From the Frobenius matrix to Q(T) and point counts (oracle; tests only).

Section 2.1: Z(X,T) = Q(T)^((-1)^n) / prod_{i<n} (1 - p^i T) with
Q(T) = det(1 - T Phi), Phi the matrix of p^{-1} sigma on H^n_dR(U).
With Phi' the matrix whose column c holds the coordinates of
p^{m_c-n-1} sigma(x^beta Omega / f^{m_c}) (Proposition 2.1), Phi = Phi' diag(p^(n-m_c)).

The integer recovery follows the Weil bounds (|alpha| = p^(w/2), w = n-1) and
Mazur's Newton-over-Hodge divisibility (Section 2.5), with the functional
equation a_{b-i} = (-1)^b det(Phi') p^(w(b-2i)/2) a_i.
"""
from fractions import Fraction
from math import comb

import numpy as np


def symlift(x, m):
    x %= m
    return x - m if 2 * x > m else x


def charpoly_coeffs(A):
    """Exact det(I - T A) coefficients [1, c_1, ..., c_b] (Faddeev-LeVerrier)."""
    b = len(A)
    A = [[int(x) for x in row] for row in A]
    c = [1]
    Mk = [[0] * b for _ in range(b)]  # M_0 = 0
    for k in range(1, b + 1):
        # M_k = A M_{k-1} + c_{k-1} I
        AM = [[sum(A[i][t] * Mk[t][j] for t in range(b)) for j in range(b)] for i in range(b)]
        for i in range(b):
            AM[i][i] += c[k - 1]
        Mk = AM
        tr = sum(sum(A[i][t] * Mk[t][i] for t in range(b)) for i in range(b))
        assert tr % k == 0
        c.append(-tr // k)
    return c


def power_sums(A, kmax):
    b = len(A)
    A = [[int(x) for x in row] for row in A]
    P = [[int(i == j) for j in range(b)] for i in range(b)]
    out = []
    for _ in range(kmax):
        P = [[sum(P[i][t] * A[t][j] for t in range(b)) for j in range(b)] for i in range(b)]
        out.append(sum(P[i][i] for i in range(b)))
    return out


def det_exact(A):
    b = len(A)
    M = [[Fraction(int(x)) for x in row] for row in A]
    det = Fraction(1)
    for c in range(b):
        piv = next((r for r in range(c, b) if M[r][c] != 0), None)
        if piv is None:
            return 0
        if piv != c:
            M[c], M[piv] = M[piv], M[c]
            det = -det
        det *= M[c][c]
        for r in range(c + 1, b):
            f = M[r][c] / M[c][c]
            if f:
                for k in range(c, b):
                    M[r][k] -= f * M[c][k]
    return int(det)


def _gt(p, e, scale, i, w):
    return p ** (2 * e) > scale * scale * p ** (i * w)


def recover_lpoly(phi_prime, col_pole, p, n, r):
    """Integer Q(T) from Phi' (any integer lift of its residues, known mod p^r
    or better in every column).  Returns (coeffs a_0..a_b, sign eps')."""
    b = len(phi_prime)
    w = n - 1
    slope = [n - m for m in col_pole]
    slopes = sorted(slope)
    mu = slopes[0]
    Phi = [[int(phi_prime[i][j]) * p ** slope[j] for j in range(b)] for i in range(b)]
    c = charpoly_coeffs(Phi)
    ps = power_sums(Phi, b // 2)
    a = [1] + [None] * b
    s = []
    for i in range(1, b // 2 + 1):
        h_i = sum(slopes[:i])
        if _gt(p, r + h_i, 2 * comb(b, i), i, w):
            a[i] = symlift(c[i], p ** (r + h_i))
            s.append(-i * a[i] - sum(s[k - 1] * a[i - k] for k in range(1, i)))
        elif _gt(p, r + i * mu, 2 * b, i, w):
            s_i = symlift(ps[i - 1], p ** (r + i * mu))
            s.append(s_i)
            num = -sum(s[k - 1] * a[i - k] for k in range(1, i + 1))
            if num % i:
                raise ArithmeticError("Newton identity not integral at i=%d" % i)
            a[i] = num // i
        else:
            raise ArithmeticError("precision r=%d too small for a_%d" % (r, i))
    d0 = det_exact(phi_prime) % p
    if d0 == 1:
        eps = 1
    elif d0 == p - 1:
        eps = -1
    else:
        raise ArithmeticError("det Phi' = %d mod p is not +-1" % d0)
    sgn = (-1) ** b * eps
    for i in range(0, (b + 1) // 2):
        e2 = w * (b - 2 * i)
        assert e2 % 2 == 0
        a[b - i] = sgn * p ** (e2 // 2) * a[i]
    if b % 2 == 0:
        if sgn == -1 and a[b // 2] != 0:
            raise ArithmeticError("functional equation forces a_{b/2} = 0")
    return a, eps


def lpoly_power_sums(a, kmax):
    """s_k = sum alpha^k from Q(T) = sum a_i T^i (Newton's identities)."""
    s = []
    for k in range(1, kmax + 1):
        ak = a[k] if k < len(a) else 0
        s.append(-k * ak - sum(s[i - 1] * (a[k - i] if k - i < len(a) else 0) for i in range(1, k)))
    return s


def point_counts_from_lpoly(a, p, n, kmax):
    """#X(F_{p^k}) = sum_{i<n} p^(ik) + (-1)^(n+1) s_k   (Section 2.1)."""
    s = lpoly_power_sums(a, kmax)
    return [sum(p ** (i * k) for i in range(n)) + (-1) ** (n + 1) * s[k - 1]
            for k in range(1, kmax + 1)]


def weil_root_check(a, p, w, rtol=1e-6):
    """Every root alpha of T^b Q(1/T) has |alpha| = p^(w/2)."""
    coeffs = [float(x) for x in a]  # a_0 .. a_b: alpha are roots of sum a_i x^(b-i)
    roots = np.roots(coeffs)
    target = float(p) ** (w / 2.0)
    return bool(np.all(np.abs(np.abs(roots) / target - 1.0) < rtol))


def _poly_divmod(num, den):
    """Quotient and remainder of polynomials over Q (coefficient lists, lowest
    degree first, Fractions)."""
    num = list(num)
    q = [Fraction(0)] * max(1, len(num) - len(den) + 1)
    while len(num) >= len(den) and any(num):
        k = len(num) - len(den)
        c = num[-1] / den[-1]
        q[k] = c
        for i, d in enumerate(den):
            num[i + k] -= c * d
        num.pop()
        while num and num[-1] == 0:
            num.pop()
    return q, num


def squarefree_part(a):
    """Q / gcd(Q, Q') over Q: the same roots, each once (exact, Fractions)."""
    f = [Fraction(x) for x in a]
    while f and f[-1] == 0:
        f.pop()
    df = [i * f[i] for i in range(1, len(f))]
    g, h = f, df
    while h and any(h):
        _, r = _poly_divmod(g, h)
        g, h = h, r
    q, r = _poly_divmod(f, g)
    assert not any(r)
    return q


def weil_root_check_squarefree(a, p, w, rtol=1e-6):
    """weil_root_check on the squarefree part of Q(T): repeated roots (common
    on the algebraic classes of a surface, alpha = p times a root of unity)
    are found to only about a cube root of the working precision by a
    numerical root finder; removing the repetition first keeps the check
    within rtol."""
    sq = squarefree_part(a)
    lead = sq[0]
    return weil_root_check([x / lead for x in sq], p, w, rtol)
