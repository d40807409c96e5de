"""Newton-polygon invariants (Sections 1.2, 6.3, 6.4, 6.6): the oracle's
definitions pinned by polynomials with roots of known valuation and by closed
forms of Fermat hypersurfaces (Weil's Gauss-sum formula; supersingular
Fermat curves), and the paper's fact that the Fermat quintic surface is
ordinary over F_11 (Section 6.4); the library's cr_newton_polygon (host only)
against the oracle on the same polynomials."""
import json
import os
from fractions import Fraction

import pytest

from oracle.diagonal import fermat_coeffs, fermat_lpoly
from oracle.frobenius import frobenius
from oracle.newton import invariants, newton_slopes
from paper_2602_24155_amd import crfrob as C

HERE = os.path.dirname(os.path.abspath(__file__))


def expand(factors):
    """Coefficients of prod (1 + c_1 T + ... + c_k T^k) over the factor lists."""
    out = [1]
    for f in factors:
        nxt = [0] * (len(out) + len(f))
        for i, a in enumerate(out):
            nxt[i] += a
            for j, c in enumerate(f):
                nxt[i + j + 1] += a * c
        out = nxt
    return out


def hodge_of(nv, d):
    n = nv - 1
    from math import comb
    return {m: sum((-1) ** j * comb(nv, j) * comb(d * m - n - 1 - j * (d - 1) + n, n)
                   for j in range(nv) if d * m - n - 1 - j * (d - 1) >= 0) for m in range(1, n + 1)}


def test_slopes_of_products_with_known_valuations():
    p = 7
    # roots alpha = unit * p^k give slope k; 1 + p^a T^2 (irreducible over Q_p when a is odd) slope a/2 twice
    a = expand([[-3], [-5 * p], [2 * p], [-p ** 2], [p ** 3]])
    assert newton_slopes(a, p) == [(0, 1), (1, 2), (2, 1), (3, 1)]
    a = expand([[0, p]] * 3)
    assert newton_slopes(a, p) == [(Fraction(1, 2), 6)]
    a = expand([[-p], [0, p ** 3], [-4]])
    assert newton_slopes(a, p) == [(0, 1), (1, 1), (Fraction(3, 2), 2)]


def test_fermat_quartic_curve_supersingular_at_7():
    a = fermat_lpoly(3, 4, 7)  # (1 + 7 T^2)^3, d | p + 1
    assert a == expand([[0, 7]] * 3)
    inv = invariants(a, 7, 2, hodge_of(3, 4))
    assert inv["supersingular"] and inv["p_rank"] == 0 and not inv["ordinary"]


@pytest.mark.parametrize("p", [11, 31, 41])
def test_fermat_quintic_curve_ordinary_when_5_divides_p_minus_1(p):
    inv = invariants(fermat_lpoly(3, 5, p), p, 2, hodge_of(3, 5))
    assert inv["ordinary"] and inv["p_rank"] == 6 and not inv["supersingular"]


def test_fermat_quartic_k3_heights():
    """p = 1 mod 4: ordinary (height 1, Hodge-Witt); p = 3 mod 4: supersingular
    (height infinite, domino 1); Section 6.3 and the K3 remark of Section 1.2."""
    inv = invariants(fermat_lpoly(4, 4, 13), 13, 3, hodge_of(4, 4))
    assert inv["ordinary"] and inv["height"] == 1 and inv["domino"] == 0
    for p in (7, 11):
        a = frobenius(4, 4, p, fermat_coeffs(4, 4)).lpoly
        inv = invariants(a, p, 3, hodge_of(4, 4))
        assert inv["supersingular"] and inv["height"] == float("inf") and inv["domino"] == 1


def test_fermat_quintic_surface_ordinary_at_11():
    """Section 6.4: the Fermat quintic surface is ordinary in characteristic 11,
    so Hodge-Witt (domino number 0); its Q(T) from Weil's formula."""
    facts = json.load(open(os.path.join(HERE, "golden", "paper_facts.json")))["newton"]
    e = [f for f in facts if f["family"] == "Fermat quintic surface" and f["p"] == 11][0]
    a = fermat_lpoly(4, 5, 11)
    inv = invariants(a, 11, 3, hodge_of(4, 5))
    assert inv["ordinary"] == e["ordinary"] and inv["domino"] == 0 and inv["p_rank"] == 4


def _lib(nv, d, p, a):
    words = C.lpoly_words(a)
    return C.cr_newton_polygon(nv, d, p, words)


def _same(lib, inv):
    slopes = [(Fraction(r, ln), ln) for ln, r in zip(lib.seg_len[:lib.nseg], lib.seg_rise[:lib.nseg])]
    assert slopes == inv["slopes"]
    assert lib.p_rank == inv["p_rank"]
    assert bool(lib.ordinary) == inv["ordinary"] and bool(lib.supersingular) == inv["supersingular"]
    h = inv["height"]
    assert lib.height == (-1 if h is None else (0 if h == float("inf") else int(h)))
    dm = inv["domino"]
    assert (lib.domino_num, lib.domino_den) == ((-1, 1) if dm is None else (dm.numerator, dm.denominator))


@pytest.mark.parametrize("nv,d,p", [(3, 4, 7), (3, 5, 11), (3, 5, 19), (4, 4, 13), (4, 5, 11)])
def test_library_matches_oracle_on_closed_forms(nv, d, p):
    a = fermat_lpoly(nv, d, p)
    _same(_lib(nv, d, p, a), invariants(a, p, nv - 1, hodge_of(nv, d)))


def test_library_matches_oracle_on_k3_goldens():
    gold = json.load(open(os.path.join(HERE, "golden", "k3_golden.json")))["items"]
    for g in gold:
        a = [int(x) for x in g["lpoly"]]
        inv = invariants(a, g["p"], 3, hodge_of(4, 4))
        assert inv["height"] is not None and inv["domino"] in (0, 1)
        _same(_lib(4, 4, g["p"], a), inv)


def test_library_rejects_bad_polynomials():
    a = [2] + [0] * 21
    res = C.cr_newton_polygon(4, 4, 7, C.lpoly_words(a), raise_on_error=False)
    assert res is None
