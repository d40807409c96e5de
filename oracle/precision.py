"""Precision rule of the oracle (Section 2.5; test infrastructure only).

The paper fixes M = max_m { r_m + v_p((p s_m - 1)!) - m + 1 } with
s_m = N_m + m - 1, but leaves r_m and N_m to cited results it does not print.
Reading used here (and documented with the library): one relative precision r
for all columns, chosen so that every coefficient a_i, i <= floor(b/2), of
Q(T) is recovered either from its own congruence (a_i is known mod
p^(r + h_i), |a_i| <= C(b,i) p^(i w / 2)) or from the power sum
s_i = tr(Phi^i) (known mod p^(r + i mu), |s_i| <= b p^(i w / 2)), and
N_m = r + 1.  h_i is the Hodge polygon (sum of the i smallest column slopes
n - m), mu the smallest slope, w = n - 1 the weight.

parity unpinned as a formula (the paper prints one datum only: modulus 11^8 for
cubic threefolds over F_11); pinned by tests that the recovered Q(T) matches
brute-force point counts and that one more series term changes nothing.
"""
from math import comb, isqrt


def vp_factorial(x, p):
    """p-adic valuation of x!"""
    v, t = 0, p
    while t <= x:
        v += x // t
        t *= p
    return v


def _gt_bound(p, e, scale, i, w):
    """p^e > scale * p^(i w / 2), decided exactly (p^(i w) may be a non-square)."""
    # compare p^(2e) > scale^2 * p^(i w)
    return p ** (2 * e) > scale * scale * p ** (i * w)


def relative_precision(p, n, hodge_sizes):
    """Uniform relative precision r for a hypersurface in P^n.

    hodge_sizes[m] = |B_m| for m = 1..n."""
    b = sum(hodge_sizes.values())
    w = n - 1
    slopes = sorted(n - m for m in hodge_sizes for _ in range(hodge_sizes[m]))
    mu = slopes[0]
    r = 1
    for i in range(1, b // 2 + 1):
        h_i = sum(slopes[:i])
        rc = 1
        while not _gt_bound(p, rc + h_i, 2 * comb(b, i), i, w):
            rc += 1
        rp = 1
        while not _gt_bound(p, rp + i * mu, 2 * b, i, w):
            rp += 1
        r = max(r, min(rc, rp))
    return r


def precision_parameters(p, n, hodge_sizes, r=None, N=None):
    """(r, {m: N_m}, {m: s_m}, M) per Section 2.5 under the reading above."""
    if r is None:
        r = relative_precision(p, n, hodge_sizes)
    ms = [m for m in range(1, n + 1) if hodge_sizes.get(m, 0) > 0]
    Nm = {m: (N[m] if isinstance(N, dict) else (N if N is not None else r + 1)) for m in ms}
    sm = {m: Nm[m] + m - 1 for m in ms}
    M = max(r + vp_factorial(p * sm[m] - 1, p) - m + 1 for m in ms)
    return r, Nm, sm, M


__all__ = ["vp_factorial", "relative_precision", "precision_parameters", "isqrt"]
