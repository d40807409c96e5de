"""The oracle's Frobenius matrix (test infrastructure only).

Steps, in the paper's order:

1. validate p and the S-smoothness of the lift f (Definition 3.1);
2. monomial basis B_m, m = 1..n (Section 2.3);
3. precision r, N_m, s_m, M (Section 2.5; rule in ``precision.py``);
4. Frobenius start terms (Proposition 2.1): for a basis element x^beta/f^m,
   j < N_m and |alpha| = dj the term
       p^(m-1) D_{j,m} C_{j,alpha} x^(p(beta+alpha+1)) Omega / (f^(p(m+j)) x^1)
   with D_{j,m} = sum_{i=j}^{N_m-1} (-1)^(i+j) binom(-m,i) binom(i,j) and
   C_{j,alpha} the coefficient of x^alpha in f^j.  The p^(m-1) is kept out and
   each term is pre-multiplied by (p s_m - 1)!/(P - 1)!, P = p(m+j), so that
   reducing without dividing by the pole orders multiplies every term by the
   same (p s_m - 1)!/(n-1)!.
   In the x^S form of Proposition 3.3 the numerator exponent is
   E' = p(beta+alpha+1) - 1 + 1_S; terms of one column with equal E' are added.
5. controlled reduction to pole n, one pole order per step (Proposition 3.3,
   explicit R_{u,v} of Section 3.1, Tweak of Algorithm 1, greedy v of
   Algorithm 3) -- in ``oracle_c.c``;
6. Griffiths-Dwork reduction of the pole-n numerators to the basis
   (Section 3.3 step (2));
7. per-column unscaling: divide by the unit part of (p s_m - 1)!/(n-1)! and
   exactly by p^(v_p((p s_m - 1)!) - m + 1); the column is then known mod
   p^(M - v_p((p s_m - 1)!) + m - 1) >= p^r.
"""
from dataclasses import dataclass, field
from math import comb, factorial

import numpy as np

from . import _native
from .cohomology import basis, gd_coordinates, is_s_smooth, psi_matrix
from .lpoly import recover_lpoly
from .poly import from_coeffs, index_of, monomials, pmul
from .precision import precision_parameters, vp_factorial


def is_prime(p):
    return p >= 2 and all(p % k for k in range(2, int(p ** 0.5) + 1))


def binom_neg(m, i):
    """binom(-m, i) = (-1)^i binom(m+i-1, i)."""
    return (-1) ** i * comb(m + i - 1, i)


def d_coeff(j, m, N):
    """D_{j,m} of Proposition 2.1 (index reading: the sum runs over i = j..N-1)."""
    return sum((-1) ** (i + j) * binom_neg(m, i) * comb(i, j) for i in range(j, N))


@dataclass
class OracleResult:
    p: int
    n: int
    d: int
    S: list
    r: int
    N: dict
    M: int
    q: int
    basis: dict
    col_pole: list
    scaled: np.ndarray          # b x b, Y = coords of the reduced sums, mod p^M
    phi_prime: list             # b x b ints, column c known mod p^(col_prec[c])
    col_prec: list
    lpoly: list = None
    eps: int = None
    nblocks: int = 0
    steps: int = 0
    extra: dict = field(default_factory=dict)


def start_blocks(f, nv, d, p, S, B, Nm, sm, q):
    """Proposition 2.1 terms grouped by numerator exponent E' (x^S form).

    Returns (list of E' tuples, list of poles, coefficient matrix nblk x b mod q,
    column pole list)."""
    n = nv - 1
    cols = [(m, beta) for m in range(1, n + 1) for beta in B[m]]
    b = len(cols)
    Jmax = max(Nm.values())
    fpow = [{(0,) * nv: 1}]
    for _ in range(1, Jmax):
        fpow.append(pmul(fpow[-1], f))
    blocks = {}
    for c, (m, beta) in enumerate(cols):
        N = Nm[m]
        top = factorial(p * sm[m] - 1)
        for j in range(N):
            Djm = d_coeff(j, m, N)
            if Djm == 0:
                continue
            P = p * (m + j)
            scale = top // factorial(P - 1)
            for alpha, C in fpow[j].items():
                E = tuple(p * (beta[i] + alpha[i] + 1) - 1 + (1 if i in S else 0) for i in range(nv))
                if E not in blocks:
                    blocks[E] = (P, [0] * b)
                assert blocks[E][0] == P
                row = blocks[E][1]
                row[c] = (row[c] + Djm * C * scale) % q
    keys = sorted(blocks, key=lambda e: (-blocks[e][0], tuple(-x for x in e)))
    E = [k for k in keys]
    P = [blocks[k][0] for k in keys]
    coef = np.array([blocks[k][1] for k in keys], dtype=object).reshape(len(keys), b)
    return E, P, coef, [m for (m, _beta) in cols]


def reduce_blocks(f, nv, d, p, S, q, E, P, coef, check_identity=False):
    """Pole-n numerators H = sum_blocks coef x (reduced numerator), mod q."""
    n = nv - 1
    Smask = sum(1 << i for i in S)
    psi, src, tmon, J = psi_matrix(f, nv, d, S, q, p)
    gmon = monomials(nv, d * n - n)
    fmon = monomials(nv, d * n - n - 1)
    b = coef.shape[1]
    H = np.zeros((len(fmon), b), dtype=np.uint64)
    if len(E) == 0:
        return H, 0
    sexp = _native.i32([mu for (_i, mu) in src])
    sblk = _native.i32([i for (i, _mu) in src])
    gexp = _native.i32(gmon)
    texp = _native.i32(tmon)
    fexp = _native.i32(fmon)
    Ex = _native.i32(E)
    Px = _native.i32(P)
    co = _native.u64(np.asarray(coef, dtype=object) % q)
    psi = _native.u64(psi)
    Jc = _native.u64(np.asarray(J, dtype=object) % q) if check_identity else None
    L = _native.lib()
    rc = L.orc_reduce(nv, d, Smask, q,
                      len(gmon), _native.ptr_i32(gexp), len(tmon), _native.ptr_i32(texp),
                      len(src), _native.ptr_i32(sexp), _native.ptr_i32(sblk),
                      _native.ptr_u64(psi), len(fmon), _native.ptr_i32(fexp),
                      len(E), _native.ptr_i32(Ex), _native.ptr_i32(Px), b,
                      _native.ptr_u64(co), _native.ptr_u64(H),
                      _native.ptr_u64(Jc) if Jc is not None else None)
    if rc != 0:
        raise RuntimeError("orc_reduce failed with code %d" % rc)
    steps = sum(pp - n for pp in P)
    return H, steps


def frobenius(nv, d, p, coeffs, S=None, r=None, N=None, M=None, lpoly=True,
              check_identity=False, columns=None):
    """Frobenius data of the hypersurface with integer coefficients ``coeffs``
    (lex-descending monomial order; any integer lift of the F_p coefficients).

    r, N, M override the precision rule (N may be an int or {m: N_m}).
    ``columns`` restricts the computation to a subset of basis columns (exact
    for those columns, since columns never mix)."""
    n = nv - 1
    if not is_prime(p):
        raise ValueError("p must be prime")
    if not (7 <= p < 50) or p <= n or d % p == 0:
        raise ValueError("need 7 <= p < 50, p > n, p not dividing d")
    S = sorted(range(nv)) if S is None else sorted(S)
    if d < len(S):
        raise ValueError("controlled reduction needs d >= |S|")
    f = from_coeffs(nv, d, coeffs)
    fp = {e: c % p for e, c in f.items() if c % p}
    if not is_s_smooth(fp, nv, d, p, sorted(range(nv))):
        raise ValueError("singular")
    if not is_s_smooth(fp, nv, d, p, S):
        raise ValueError("not S-smooth")
    B = basis(fp, nv, d, p)
    sizes = {m: len(B[m]) for m in B}
    r0, Nm, sm, M0 = precision_parameters(p, n, sizes, r=r, N=N)
    Mw = M0 if M is None else M
    q = p ** Mw
    if q >= 1 << 62:
        raise ValueError("p^M too large for the oracle's 64-bit residues")
    E, P, coef, col_pole = start_blocks(f, nv, d, p, S, B, Nm, sm, q)
    if columns is not None:
        mask = np.zeros(coef.shape[1], dtype=bool)
        mask[list(columns)] = True
        coef = coef * mask
        # start terms whose coefficients in the kept columns are all zero add nothing
        keep = [k for k in range(len(E)) if any(int(x) for x in coef[k])]
        E, P, coef = [E[k] for k in keep], [P[k] for k in keep], coef[keep, :]
    H, steps = reduce_blocks(f, nv, d, p, S, q, E, P, coef, check_identity=check_identity)
    Y = gd_coordinates(f, nv, d, p, q, B, H.astype(object))
    b = len(col_pole)
    phi = [[0] * b for _ in range(b)]
    col_prec = []
    for c in range(b):
        m = col_pole[c]
        v = vp_factorial(p * sm[m] - 1, p)
        F = factorial(p * sm[m] - 1) // factorial(n - 1)
        unit = F // p ** v
        shift = v - (m - 1)
        prec = Mw - shift
        col_prec.append(prec)
        inv = pow(unit, -1, p ** prec)
        for i in range(b):
            y = int(Y[i, c])
            if y % p ** shift:
                raise ArithmeticError("column %d not divisible by p^%d: series order or "
                                      "precision too small" % (c, shift))
            phi[i][c] = (y // p ** shift) * inv % p ** prec
    res = OracleResult(p=p, n=n, d=d, S=S, r=r0, N=Nm, M=Mw, q=q, basis=B,
                       col_pole=col_pole, scaled=Y, phi_prime=phi, col_prec=col_prec,
                       nblocks=len(E), steps=steps)
    if lpoly and columns is None:
        res.lpoly, res.eps = recover_lpoly(phi, col_pole, p, n, r0)
    return res
