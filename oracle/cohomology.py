"""Griffiths-Dwork cohomology pieces of the oracle (test infrastructure only).

* S-smoothness (Definition 3.1): J_S = <d_i f>_{i in S} + <x_i d_i f>_{i not in S}
  defines the empty scheme iff it is surjective onto Homog_D with
  D = dn + d - n - |S| (Macaulay's bound; for S = all this is the Jacobian
  criterion in degree (n+1)(d-2)+1).
* Monomial basis (Section 2.3): for m = 1..n, the monomials of degree
  k = dm-n-1 that are NOT pivot columns of the row-echelon form mod p of the
  image of M_k, columns scanned in lex-descending monomial order.
* The decomposition map of Proposition 3.3: a right inverse psi of J_S over
  Z/p^M.
* The final Griffiths-Dwork reduction (Section 3.3 step (2), relation (1)):
  h = sum_{beta in B_m} c_beta x^beta + sum_i a_i d_i f at pole m, then
  continue with (1/(m-1)) sum_i d_i a_i at pole m-1.
"""
import numpy as np

from . import _native
from .poly import index_of, monomials, pderiv, pmul


def smask_set(nv, S):
    return sorted(range(nv)) if S is None else sorted(S)


def rank_pivots_mod_p(rows, p):
    """Row-reduce an integer matrix mod p; return the pivot column list."""
    A = np.array(rows, dtype=np.int64) % p
    if A.size == 0:
        return []
    nr, nc = A.shape
    piv = []
    r = 0
    for c in range(nc):
        if r == nr:
            break
        nzr = np.nonzero(A[r:, c])[0]
        if nzr.size == 0:
            continue
        s = r + int(nzr[0])
        if s != r:
            A[[r, s]] = A[[s, r]]
        inv = pow(int(A[r, c]), -1, p)
        A[r] = (A[r] * inv) % p
        col = A[:, c].copy()
        col[r] = 0
        A = (A - np.outer(col, A[r])) % p
        piv.append(c)
        r += 1
    return piv


def jacobian_generators(f, nv, d, S, D):
    """Columns of J_S into Homog_D: list of (block i, multiplier mu, polynomial)."""
    gens = []
    for i in range(nv):
        di = pderiv(f, i)
        if i in S:
            base, mdeg = di, D - d + 1
        else:
            xi = tuple(1 if j == i else 0 for j in range(nv))
            base, mdeg = pmul({xi: 1}, di), D - d
        for mu in monomials(nv, mdeg):
            gens.append((i, mu, pmul({mu: 1}, base)))
    return gens


def js_degree(nv, d, S):
    n = nv - 1
    return d * n + d - n - len(S)


def is_s_smooth(f, nv, d, p, S):
    D = js_degree(nv, d, S)
    tmon = monomials(nv, D)
    tidx = index_of(tmon)
    rows = []
    for (_i, _mu, g) in jacobian_generators(f, nv, d, S, D):
        v = [0] * len(tmon)
        for e, c in g.items():
            v[tidx[e]] = c % p
        rows.append(v)
    return len(rank_pivots_mod_p(rows, p)) == len(tmon)


def basis(f, nv, d, p):
    """B_m for m = 1..n (Section 2.3); returns {m: [exponent tuples]}."""
    n = nv - 1
    out = {}
    for m in range(1, n + 1):
        k = d * m - n - 1
        kmon = monomials(nv, k)
        if not kmon:
            out[m] = []
            continue
        kidx = index_of(kmon)
        rows = []
        for i in range(nv):
            di = pderiv(f, i)
            for mu in monomials(nv, k - d + 1):
                g = pmul({mu: 1}, di)
                v = [0] * len(kmon)
                for e, c in g.items():
                    v[kidx[e]] = c % p
                rows.append(v)
        piv = set(rank_pivots_mod_p(rows, p)) if rows else set()
        out[m] = [kmon[j] for j in range(len(kmon)) if j not in piv]
    return out


def psi_matrix(f, nv, d, S, q, p):
    """Right inverse psi (src x tgt) of J_S over Z/q and the src/tgt layouts."""
    D = js_degree(nv, d, S)
    tmon = monomials(nv, D)
    tidx = index_of(tmon)
    gens = jacobian_generators(f, nv, d, S, D)
    J = np.zeros((len(tmon), len(gens)), dtype=object)
    for col, (_i, _mu, g) in enumerate(gens):
        for e, c in g.items():
            J[tidx[e], col] = c % q
    psi, rank = _native.right_inverse(J, q, p)
    if rank != len(tmon):
        raise ValueError("f is not S-smooth mod p")
    src = [(i, mu) for (i, mu, _g) in gens]
    return psi, src, tmon, J


def matmul_mod(A, B, q):
    return (np.asarray(A, dtype=object).dot(np.asarray(B, dtype=object))) % q


def gd_coordinates(f, nv, d, p, q, B, H):
    """Coordinates in the basis of the pole-n forms with numerators H.

    H: (dim Homog_{dn-n-1}) x b integer matrix (one form per column).
    Returns a (sum_m |B_m|) x b matrix over Z/q; rows follow the basis order
    (m = 1..n, then B_m order)."""
    n = nv - 1
    H = np.asarray(H, dtype=object) % q
    coords = {}
    for m in range(n, 0, -1):
        k = d * m - n - 1
        kmon = monomials(nv, k)
        kidx = index_of(kmon)
        gens = []
        for i in range(nv):
            di = pderiv(f, i)
            for mu in monomials(nv, k - d + 1):
                gens.append((i, mu, pmul({mu: 1}, di)))
        ncol = len(gens) + len(B[m])
        A = np.zeros((len(kmon), ncol), dtype=object)
        for col, (_i, _mu, g) in enumerate(gens):
            for e, c in g.items():
                A[kidx[e], col] = c % q
        for j, beta in enumerate(B[m]):
            A[kidx[beta], len(gens) + j] = 1
        if len(kmon) == 0:
            coords[m] = np.zeros((0, H.shape[1]), dtype=object)
            continue
        X, rank = _native.right_inverse(A, q, p)
        if rank != len(kmon):
            raise ValueError("basis does not complete the image at pole %d" % m)
        sol = matmul_mod(X.astype(object), H, q)
        coords[m] = sol[len(gens):, :]
        if m == 1:
            break
        # h' = (1/(m-1)) sum_i d_i a_i at pole m-1
        k2 = d * (m - 1) - n - 1
        k2mon = monomials(nv, k2)
        k2idx = index_of(k2mon)
        Hn = np.zeros((len(k2mon), H.shape[1]), dtype=object)
        inv = pow(m - 1, -1, q)
        for row, (i, mu, _g) in enumerate(gens):
            if mu[i] == 0:
                continue
            e = list(mu)
            e[i] -= 1
            Hn[k2idx[tuple(e)], :] += mu[i] * sol[row, :]
        H = (Hn * inv) % q
    return np.vstack([coords[m] for m in range(1, n + 1)])
