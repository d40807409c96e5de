"""Pins of the CPU oracle against facts independent of it.

* Weil's Gauss-sum formula / supersingular closed forms for Fermat
  hypersurfaces (whole Q(T));
* brute-force #X(F_{p^k}) (Section 1.1 definition of Z(X,T));
* invariance of Q(T) under the lift of f and under permuting variables (the
  Frobenius matrix changes, Q(T) may not);
* Riemann hypothesis |alpha| = p^((n-1)/2), det Phi' = +-1 mod p;
* convergence: one more Frobenius series term does not change Phi' mod p^r;
* the paper's precision datum (modulus 11^8 for cubic threefolds over F_11,
  Section 5.3);
* elementary identities: D_{j,m} (Proposition 2.1), Hodge numbers, the
  decomposition identity of Proposition 3.3 at every step, and that the
  Griffiths-Dwork coordinates vanish on the Jacobian ideal.
"""
from math import comb

import numpy as np
import pytest

from oracle import frobenius as ofrob
from oracle.cohomology import basis, gd_coordinates
from oracle.diagonal import fermat_coeffs, fermat_lpoly
from oracle.frobenius import d_coeff, frobenius
from oracle.lpoly import point_counts_from_lpoly, weil_root_check
from oracle.poly import from_coeffs, monomials, pderiv, pmul, index_of
from oracle.pointcount import count_projective
from oracle.precision import precision_parameters
from paper_2602_24155_amd import workload


def _random_smooth(nv, d, p, seed):
    rng = np.random.default_rng(seed)
    while True:
        c = [int(x) for x in rng.integers(0, p, size=comb(d + nv - 1, nv - 1))]
        try:
            return c, frobenius(nv, d, p, c)
        except ValueError:
            continue


@pytest.mark.parametrize("nv,d,p", [(3, 4, 7), (3, 4, 13), (3, 4, 11), (3, 5, 11), (3, 5, 19),
                                    (3, 5, 31), (3, 5, 41), (4, 4, 13)])
def test_fermat_closed_form(nv, d, p):
    res = frobenius(nv, d, p, fermat_coeffs(nv, d))
    assert res.lpoly == fermat_lpoly(nv, d, p)


@pytest.mark.parametrize("nv,d,p,kmax,seed", [(3, 4, 7, 3, 1), (3, 4, 7, 3, 2), (3, 4, 11, 2, 3),
                                              (3, 5, 11, 3, 4), (3, 5, 31, 2, 5), (3, 5, 47, 1, 6),
                                              (3, 5, 13, 2, 7)])
def test_random_curve_point_counts(nv, d, p, kmax, seed):
    c, res = _random_smooth(nv, d, p, seed)
    f = from_coeffs(nv, d, c)
    brute = [count_projective(f, nv, p, k) for k in range(1, kmax + 1)]
    assert point_counts_from_lpoly(res.lpoly, p, nv - 1, kmax) == brute
    assert weil_root_check(res.lpoly, p, nv - 2)
    assert res.eps == 1  # curves: det(Phi') = 1


def test_quartic_curve_whole_lpoly_from_counts():
    # genus 3: #C(F_{7^k}), k = 1..3, fix s_1..s_3 and hence the whole L-polynomial
    p, c = workload.first_accepted("quartic_curve_f7", 0, lambda p, c: _smooth(3, 4, p, c))
    res = frobenius(3, 4, p, c)
    f = from_coeffs(3, 4, c)
    counts = [count_projective(f, 3, p, k) for k in (1, 2, 3)]
    s = [1 + p ** k - counts[k - 1] for k in (1, 2, 3)]
    a = [1]
    for k in (1, 2, 3):
        a.append(-(sum(s[i - 1] * a[k - i] for i in range(1, k + 1))) // k)
    full = a + [p ** (3 - i) * a[i] for i in (2, 1, 0)]
    assert res.lpoly == full


def _smooth(nv, d, p, c):
    from oracle.cohomology import is_s_smooth
    f = {e: v % p for e, v in from_coeffs(nv, d, c).items() if v % p}
    return is_s_smooth(f, nv, d, p, list(range(nv)))


def test_lift_invariance():
    c, res = _random_smooth(3, 4, 7, 11)
    rng = np.random.default_rng(0)
    c2 = [x + 7 * int(rng.integers(-3, 4)) for x in c]
    res2 = frobenius(3, 4, 7, c2)
    assert res2.lpoly == res.lpoly
    assert res2.phi_prime != res.phi_prime  # Phi depends on the lift; Q(T) does not


def test_permutation_invariance():
    c, res = _random_smooth(3, 5, 11, 12)
    mons = monomials(3, 5)
    idx = index_of(mons)
    perm = (2, 0, 1)
    c2 = [0] * len(mons)
    for e, v in zip(mons, c):
        c2[idx[tuple(e[perm[i]] for i in range(3))]] = v
    res2 = frobenius(3, 5, 11, c2)
    assert res2.lpoly == res.lpoly


@pytest.mark.parametrize("name,nv,d,j,subsets", [
    ("quartic_curve_f7", 3, 4, 0, [[2], [0], [1], [1, 2], [0, 2]]),
    ("quintic_curves_mixed", 3, 5, 1, [[0], [1], [1, 2], [0, 2]]),
])
def test_s_subsets_give_the_s_all_result(name, nv, d, j, subsets):
    """Definition 3.1 / Proposition 3.3 with S a proper subset: the reduction
    runs in the x^S form (sources of J_S for i not in S are x_i d_i f, the
    R_{u,v} weight of those rows is u_i + 1, Algorithm 3 forces v_i >= 1 only
    for i in S, target norm |S| - 1), but every step is still an identity in
    cohomology, so the scaled coordinates and Q(T) equal those of S = all."""
    p, c = workload.first_accepted(name, j, lambda p, c: _smooth(nv, d, p, c))
    base = frobenius(nv, d, p, c)
    from oracle.cohomology import is_s_smooth
    fp = {e: v % p for e, v in from_coeffs(nv, d, c).items() if v % p}
    ran = 0
    for S in subsets:
        if not is_s_smooth(fp, nv, d, p, S):
            with pytest.raises(ValueError):
                frobenius(nv, d, p, c, S=S)
            continue
        res = frobenius(nv, d, p, c, S=S)
        assert res.M == base.M
        assert np.array_equal(res.scaled, base.scaled), S
        assert res.lpoly == base.lpoly
        ran += 1
    assert ran >= 3


def test_s_subset_on_a_k3_column():
    """A quartic K3 surface of the stored goldens (pinned by point counts)
    reduced in the x^S form with S = {2, 3}: the m = 1 column equals the
    stored S = all column (columns never mix, so one column is exact)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "k3_golden.json")
    with open(path) as fh:
        it = [x for x in json.load(fh)["items"] if x["p"] == 7][0]
    res = frobenius(4, 4, 7, it["coeffs"], S=[2, 3], columns=[0], lpoly=False)
    assert res.col_pole[0] == 1
    assert [int(res.scaled[i][0]) for i in range(21)] == [int(row[0]) for row in it["scaled"]]


def test_convergence_one_more_term():
    c, res = _random_smooth(3, 4, 7, 13)
    r = res.r
    res2 = frobenius(3, 4, 7, c, N=r + 2, lpoly=False)
    b = len(res.col_pole)
    mod = 7 ** r
    for i in range(b):
        for j in range(b):
            assert (res.phi_prime[i][j] - res2.phi_prime[i][j]) % mod == 0


def test_precision_datum_cubic_threefold_p11():
    # cubic threefolds: Hodge numbers 0, 5, 5, 0; the paper works mod 11^8 at p = 11
    _r, _N, _s, M = precision_parameters(11, 4, {1: 0, 2: 5, 3: 5, 4: 0})
    assert M == 8


def test_d_coefficients():
    # N = 1 keeps only the leading term of the geometric series: D_{0,m} = 1
    for m in (1, 2, 3):
        assert d_coeff(0, m, 1) == 1
    # sum_j D_{j,m} t^j == sum_{i<N} binom(-m,i) (t-1)^i as polynomials in t
    for m in (1, 2, 3):
        for N in (1, 3, 6):
            lhs = [d_coeff(j, m, N) for j in range(N)]
            rhs = [0] * N
            for i in range(N):
                bi = (-1) ** i * comb(m + i - 1, i)
                for j in range(i + 1):
                    rhs[j] += bi * comb(i, j) * (-1) ** (i - j)
            assert lhs == rhs


@pytest.mark.parametrize("nv,d,p", [(3, 4, 7), (3, 5, 11), (4, 4, 7), (4, 5, 7)])
def test_hodge_numbers(nv, d, p):
    c = fermat_coeffs(nv, d)
    f = from_coeffs(nv, d, c)
    B = basis(f, nv, d, p)
    n = nv - 1
    for m in range(1, n + 1):
        k = d * m - n - 1
        # [t^k] ((1 - t^(d-1)) / (1 - t))^(n+1)
        expect = sum((-1) ** j * comb(nv, j) * comb(k - j * (d - 1) + n, n)
                     for j in range(nv) if k - j * (d - 1) >= 0)
        assert len(B[m]) == expect
    b = sum(len(v) for v in B.values())
    assert b == ((d - 1) ** nv + (-1) ** nv * (d - 1)) // d


def test_reduction_identity_checked_every_step():
    c, _ = _random_smooth(3, 4, 7, 14)
    res = frobenius(3, 4, 7, c, check_identity=True)
    assert res.steps > 0


def test_gd_coordinates_vanish_on_griffiths_dwork_relations():
    """(f d_i g - m g d_i f) Omega / f^(m+1) is exact (relation (1)): coordinates 0,
    while g d_i f Omega / f^2 alone has the coordinates of d_i g Omega / f."""
    c, _ = _random_smooth(3, 5, 11, 15)
    nv, d, p, n = 3, 5, 11, 2
    q = p ** 6
    f = from_coeffs(nv, d, c)
    fp = {e: v % p for e, v in f.items() if v % p}
    B = basis(fp, nv, d, p)
    fmon = monomials(nv, d * n - n - 1)
    fidx = index_of(fmon)
    cases = [(0, (2, 1, 0)), (1, (0, 1, 2)), (2, (1, 1, 1))]
    H = np.zeros((len(fmon), 2 * len(cases)), dtype=object)
    for col, (i, mu) in enumerate(cases):
        g = {mu: 1}
        rel = {}
        for e, v in pmul(f, pderiv(g, i)).items():
            rel[e] = rel.get(e, 0) + v
        for e, v in pmul(g, pderiv(f, i)).items():
            rel[e] = rel.get(e, 0) - v          # m = 1
            H[fidx[e], len(cases) + col] += v
        for e, v in rel.items():
            H[fidx[e], col] += v
    Y = gd_coordinates(f, nv, d, p, q, B, H % q)
    assert not np.any(Y[:, :len(cases)] % q)
    b1 = {beta: k for k, beta in enumerate(B[1])}
    for col, (i, mu) in enumerate(cases):
        want = [0] * Y.shape[0]
        for e, v in pderiv({mu: 1}, i).items():
            want[b1[e]] = v % q
        assert [int(x) for x in Y[:, len(cases) + col]] == want


def _counts_lpoly(p, c, g):
    """Whole L-polynomial of a plane curve of genus g from #C(F_{p^k}), k <= g."""
    f = from_coeffs(3, 4, c)
    counts = [count_projective(f, 3, p, k) for k in range(1, g + 1)]
    s = [1 + p ** k - counts[k - 1] for k in range(1, g + 1)]
    a = [1]
    for k in range(1, g + 1):
        a.append(-(sum(s[i - 1] * a[k - i] for i in range(1, k + 1))) // k)
    return a + [p ** (g - i) * a[i] for i in range(g - 1, -1, -1)]


@pytest.mark.parametrize("mutation", ["sign", "drop_j1", "shift_m", "no_prescale"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    """Plausible mistakes planted in the oracle break the point-count pin."""
    p, c = workload.first_accepted("quartic_curve_f7", 0, lambda p, c: _smooth(3, 4, p, c))
    want = _counts_lpoly(p, c, 3)
    good = d_coeff
    if mutation == "no_prescale":
        import oracle.frobenius as fr
        real = fr.factorial
        monkeypatch.setattr(fr, "factorial", lambda x: real(x) if x > 30 else 1)
    else:
        def bad(j, m, N):
            if mutation == "sign":
                return -good(j, m, N) if j == 1 else good(j, m, N)
            if mutation == "drop_j1":
                return 0 if j == 1 else good(j, m, N)
            return good(j, m + 1, N)
        monkeypatch.setattr(ofrob, "d_coeff", bad)
    try:
        res = frobenius(3, 4, p, c)
        assert res.lpoly != want
    except (ArithmeticError, ValueError):
        pass  # caught by the oracle's own divisibility / integrality / unit checks


def test_paper_printed_facts():
    """Values the paper prints: the 11^8 modulus and Hodge numbers (tests/golden)."""
    import json
    import os
    facts = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))
    for e in facts["precision_modulus"]:
        n = e["nvars"] - 1
        f = from_coeffs(e["nvars"], e["degree"], fermat_coeffs(e["nvars"], e["degree"]))
        B = basis(f, e["nvars"], e["degree"], e["p"])
        _r, _N, _s, M = precision_parameters(e["p"], n, {m: len(B[m]) for m in B})
        assert M == e["modulus_exponent"]
    for e in facts["hodge_numbers"]:
        nv, d = e["nvars"], e["degree"]
        n = nv - 1
        if nv <= 5:
            f = from_coeffs(nv, d, fermat_coeffs(nv, d))
            B = basis(f, nv, d, 7)
            sizes = [len(B[m]) for m in range(1, n + 1)]
        else:  # same Hilbert-function sizes as test_hodge_numbers checks against the basis
            sizes = [sum((-1) ** j * comb(nv, j) * comb(d * m - n - 1 - j * (d - 1) + n, n)
                         for j in range(nv) if d * m - n - 1 - j * (d - 1) >= 0)
                     for m in range(1, n + 1)]
        assert sum(sizes) == e["primitive_b"]
        if "h" in e:
            # primitive Hodge numbers: the middle one loses the hyperplane class for even n-1
            h = list(e["h"])
            if (n - 1) % 2 == 0:
                h[(n - 1) // 2] -= 1
            assert sizes == h[::-1] or sizes == h
        if "h02" in e:
            assert sizes[0] == e["h02"]


def test_weil_check_with_repeated_roots():
    """Q(T) with repeated reciprocal roots p, -p, p zeta (the algebraic classes of
    a surface give such factors): the squarefree form of the Weil check accepts
    it where plain numerical roots lose the precision, and still rejects a root
    of the wrong modulus."""
    from oracle.lpoly import squarefree_part, weil_root_check_squarefree
    p = 13
    a = [1]
    for f in [[1, -p]] * 3 + [[1, p]] * 2 + [[1, 0, p * p]] + [[1, -p, p * p]] * 2 + [[1, p, p * p]] * 2 + \
            [[1, -7, p * p]] * 2:
        nxt = [0] * (len(a) + len(f) - 1)
        for i, x in enumerate(a):
            for j, y in enumerate(f):
                nxt[i + j] += x * y
        a = nxt
    assert len(a) == 20 and len(squarefree_part(a)) == 11
    assert weil_root_check_squarefree(a, p, 2)
    bad = [x - (a[i - 1] if i else 0) for i, x in enumerate(a + [0])]  # times (1 - T)
    assert not weil_root_check_squarefree(bad, p, 2)
