"""Newton-polygon invariants of Q(T) (oracle; test infrastructure only).

Section 1.2: the Newton polygon of Q(T) = sum_j a_j T^j is the lower convex
hull of the points (j, v_p(a_j)); Mazur's theorem bounds it below by the
Hodge polygon.  For the middle cohomology of a hypersurface in P^n the
Hodge polygon has slope n - m with multiplicity h_m (the basis elements of
pole order m; Section 2.3), m = 1..n.  Invariants, as the paper defines them:

* p-rank: length of the Newton segment whose slope is the smallest Hodge
  slope (slope 0 for curves, slope 1 for cubic threefolds);
* ordinary: Newton polygon = Hodge polygon; supersingular: one slope w/2,
  w = n - 1 the weight;
* height (Section 6.3 for K3 surfaces, Section 6.6 for cubic fourfolds, the
  Hodge numbers 1, b-2, 1 around the middle slope w/2): the first Newton
  slope is w/2 - 1/h, h = infinity when it is w/2 (supersingular);
* domino number of a surface (Section 6.4): the least vertical distance
  between the Newton and the Hodge polygon over the slope-1 part of the
  Hodge polygon.

Written from these definitions with exact Fractions; pinned by closed forms
(Weil's formula for Fermat hypersurfaces, supersingular Fermat curves and
K3 surfaces) and by polynomials built from roots of known valuation.
"""
from fractions import Fraction


def vp(x, p):
    """p-adic valuation of a nonzero integer."""
    x = abs(int(x))
    assert x != 0
    v = 0
    while x % p == 0:
        x //= p
        v += 1
    return v


def newton_points(a, p):
    """Lower convex hull vertices of {(j, v_p(a_j)) : a_j != 0}, left to right."""
    pts = [(j, vp(c, p)) for j, c in enumerate(a) if c != 0]
    hull = []
    for q in pts:
        # drop the last vertex while it lies on or above the segment to q
        while len(hull) >= 2:
            (x1, y1), (x2, y2) = hull[-2], hull[-1]
            if (y2 - y1) * (q[0] - x1) >= (q[1] - y1) * (x2 - x1):
                hull.pop()
            else:
                break
        hull.append(q)
    return hull


def newton_slopes(a, p):
    """Slopes of the Newton polygon with multiplicity: list of (slope, length)."""
    h = newton_points(a, p)
    return [(Fraction(y2 - y1, x2 - x1), x2 - x1) for (x1, y1), (x2, y2) in zip(h, h[1:])]


def polygon_value(segments, x):
    """Height at abscissa x of the polygon from the origin with the given segments."""
    y, at = Fraction(0), 0
    for s, ln in segments:
        step = min(ln, x - at)
        if step <= 0:
            break
        y += s * step
        at += step
    return y


def hodge_segments(n, hodge):
    """Hodge polygon of the basis: slope n - m with multiplicity hodge[m], ascending."""
    return [(Fraction(n - m), hodge[m]) for m in sorted(hodge, reverse=True) if hodge[m] > 0]


def invariants(a, p, n, hodge):
    """Newton invariants of Q(T) = a for a hypersurface in P^n with basis sizes
    hodge[m], m = 1..n.  height: None when not defined for these Hodge numbers,
    float('inf') when supersingular.  domino: None unless n = 3 (a surface)."""
    b = len(a) - 1
    w = n - 1
    newt = newton_slopes(a, p)
    hod = hodge_segments(n, hodge)
    assert sum(ln for _, ln in newt) == b == sum(ln for _, ln in hod)
    smin = hod[0][0]
    p_rank = sum(ln for s, ln in newt if s == smin)
    ordinary = all(polygon_value(newt, x) == polygon_value(hod, x) for x in range(b + 1))
    supersingular = len(newt) == 1 and newt[0][0] == Fraction(w, 2)
    height = None
    mids = [(s, ln) for s, ln in hod]
    if len(mids) == 3 and mids[0][1] == 1 and mids[2][1] == 1 and mids[1][0] == Fraction(w, 2) \
            and mids[0][0] == Fraction(w, 2) - 1:
        first = newt[0][0]
        height = float("inf") if first == Fraction(w, 2) else 1 / (Fraction(w, 2) - first)
    domino = None
    if n == 3:
        x0 = sum(ln for s, ln in hod if s < 1)
        x1 = x0 + sum(ln for s, ln in hod if s == 1)
        domino = min(polygon_value(newt, x) - polygon_value(hod, x) for x in range(x0, x1 + 1))
    return {"slopes": newt, "p_rank": p_rank, "ordinary": ordinary, "supersingular": supersingular,
            "height": height, "domino": domino}
