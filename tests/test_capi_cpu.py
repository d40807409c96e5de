"""Host-only checks of the C-ABI library (no device needed).

* libcrfrob.so loads and exports every function declared in include/crfrob.h;
* the pure host entry points agree with the oracle: monomial order,
  dimensions, precision rule, smoothness decisions on a candidate stream.
"""
import os
import re

import numpy as np
import pytest

from oracle.cohomology import is_s_smooth
from oracle.poly import from_coeffs, monomials
from oracle.precision import precision_parameters
from paper_2602_24155_amd import crfrob as C
from paper_2602_24155_amd import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "crfrob.h")).read()
    declared = set(re.findall(r"^\s*(?:cr_status|const char \*|void)\s*\*?\s*(cr_\w+)\s*\(", hdr, re.M))
    assert declared, "no declarations parsed"
    L = C.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(C.EXPORTS)


@pytest.mark.parametrize("nv,d", [(3, 4), (3, 5), (4, 4), (4, 5), (6, 3), (5, 3)])
def test_monomials_and_dims(nv, d):
    mons = C.cr_monomials(nv, d)
    assert [tuple(int(x) for x in m) for m in mons] == monomials(nv, d)
    nco, s, b = C.cr_query_dims(nv, d)
    n = nv - 1
    assert s == len(monomials(nv, d * n - n))
    assert b == ((d - 1) ** nv + (-1) ** nv * (d - 1)) // d


@pytest.mark.parametrize("nv,d,p", [(3, 4, 7), (3, 5, 11), (3, 5, 31), (3, 5, 47), (4, 4, 7), (4, 4, 13),
                                    (5, 3, 11), (6, 3, 7)])
def test_precision_matches_oracle(nv, d, p):
    n = nv - 1
    hodge = {}
    for m in range(1, n + 1):
        k = d * m - n - 1
        hodge[m] = sum((-1) ** j * __import__("math").comb(nv, j) *
                       __import__("math").comb(k - j * (d - 1) + n, n)
                       for j in range(nv) if k - j * (d - 1) >= 0)
    r, Nm, _s, M = precision_parameters(p, n, hodge)
    assert C.cr_precision(C.family(nv, d), p) == (r, r + 1, M)


@pytest.mark.parametrize("name", ["quartic_curve_f7", "quintic_curves_mixed", "quartic_k3_mixed"])
def test_smoothness_agrees_with_oracle(name):
    w = workload.WORKLOADS[name]
    fam = C.family(w.nvars, w.degree)
    for j in range(3):
        p, gen = workload.stream(name, j)
        for _ in range(4):
            c = next(gen)
            f = {e: v % p for e, v in from_coeffs(w.nvars, w.degree, c).items() if v % p}
            assert C.cr_check_smooth(fam, p, c) == is_s_smooth(f, w.nvars, w.degree, p, list(range(w.nvars)))
    # a visibly singular form: x0^d
    c = [1] + [0] * (w.ncoeff - 1)
    assert not C.cr_check_smooth(fam, 7 if 7 in w.primes else w.primes[0], c)


def test_invalid_arguments_are_rejected():
    fam = C.family(3, 5)
    with pytest.raises(C.CrError) as e:
        C.cr_frobenius_batch(fam, [31], [[40] * 21])
    assert e.value.status == C.CR_EINVAL
    with pytest.raises(C.CrError) as e:
        C.cr_precision(C.family(2, 5), 31)
    assert e.value.status == C.CR_EINVAL


def test_bad_prime_statuses_without_device():
    fam = C.family(3, 5)
    # p = 9 is not prime, p = 53 is out of range: rejected by host validation
    with pytest.raises(C.CrError):
        C.cr_check_smooth(fam, 9, [1] * 21)
    with pytest.raises(C.CrError):
        C.cr_check_smooth(fam, 53, [1] * 21)


def test_family_options_are_validated():
    items = [(31, [1] * 21)]
    for kw in ({"launch": 3}, {"policy": 7}, {"engine": 6},
               {"engine": C.ENGINE_MFMA_LDS, "policy": C.CR_POLICY_P_CHUNK}):
        with pytest.raises(C.CrError) as e:
            C.cr_frobenius_batch(C.family(3, 5, **kw), [p for p, _ in items], [c for _, c in items])
        assert e.value.status == C.CR_EINVAL, kw
    with pytest.raises(C.CrError) as e:
        C.cr_autotune(C.family(3, 5), [31], [[1] * 21], trials=0)
    assert e.value.status == C.CR_EINVAL


@pytest.mark.parametrize("d", [0, 1, 2, 3, 4, 5, 6, 8])
def test_closed_form_rank_of_three_variable_monomials(d):
    """The pair kernel finds a direction's index (degree d) and a final
    exponent's index (degree |S| - 1 <= 2) by the closed form
    (d - v0)(d - v0 + 1)/2 + (d - v0 - v1); it must agree with the monomial
    order of the library (degrees it takes as a family) and of the oracle
    (every degree), which test_monomials_and_dims ties together."""
    orders = [monomials(3, d)]
    if d >= 3:
        orders.append([tuple(int(x) for x in m) for m in C.cr_monomials(3, d)])
    for mons in orders:
        for idx, m in enumerate(mons):
            r = d - m[0]
            assert r * (r + 1) // 2 + (r - m[1]) == idx


@pytest.mark.parametrize("nv,d,p", [(3, 4, 7), (3, 5, 31), (4, 4, 11)])
def test_precision_overrides_match_oracle(nv, d, p):
    """cr_family.M and cr_family.n_series_m (Section 2.5 / Proposition 2.1)
    against the oracle's precision rule with the same overrides."""
    from math import comb as _c
    n = nv - 1
    hodge = {m: sum((-1) ** j * _c(nv, j) * _c(d * m - n - 1 - j * (d - 1) + n, n)
                    for j in range(nv) if d * m - n - 1 - j * (d - 1) >= 0) for m in range(1, n + 1)}
    r, _Nm, _s, M = precision_parameters(p, n, hodge)
    nm = [r + 1 + (m % 2) for m in range(1, n + 1)]
    r2, Nm2, _s2, M2 = precision_parameters(p, n, hodge, N={m: nm[m - 1] for m in range(1, n + 1)})
    assert C.cr_precision(C.family(nv, d, n_series_m=nm), p) == (r2, max(nm), M2)
    assert C.cr_precision(C.family(nv, d, M=M + 2), p) == (r, r + 1, M + 2)
    with pytest.raises(C.CrError) as e:
        C.cr_precision(C.family(nv, d, M=M - 1), p)
    assert e.value.status == C.CR_EINVAL
    assert C.cr_residue_words(C.family(nv, d), p) == 1


def test_residue_words_reject_wide_moduli():
    # quintic surfaces over F_7 need p^M ~ 2^132: beyond the one-word residues
    with pytest.raises(C.CrError) as e:
        C.cr_residue_words(C.family(4, 5), 7)
    assert e.value.status == C.CR_EPRECISION
    with pytest.raises(C.CrError) as e:
        C.cr_residue_words(C.family(3, 5, M=40), 31)
    assert e.value.status == C.CR_EPRECISION


def test_single_hypersurface_entry_rejects_bad_input_without_device():
    with pytest.raises(C.CrError) as e:
        C.cr_frobenius(C.family(3, 5), 31, [40] * 21)
    assert e.value.status == C.CR_EINVAL
    with pytest.raises(C.CrError) as e:
        C.cr_frobenius(C.family(3, 5), 9, [1] * 21)
    assert e.value.status in (C.CR_ENOTPRIME, C.CR_EINVAL)


def test_allocator_hook_arguments_without_device():
    """cr_set_allocator: one hook without the other is CR_EINVAL; installing and
    removing hooks before any device work allocates nothing."""
    L = C.lib()
    calls = []
    alloc = C.ALLOC_FN(lambda n, ctx: calls.append(n) or None)
    assert L.cr_set_allocator(alloc, C.FREE_FN(), None) == C.CR_EINVAL
    assert L.cr_set_allocator(C.ALLOC_FN(), C.FREE_FN(lambda p, ctx: None), None) == C.CR_EINVAL
    with pytest.raises(ValueError):
        C.cr_set_allocator(alloc=lambda n: 0)
    C.cr_set_allocator(lambda n: calls.append(n) or 0, lambda ptr: None)
    C.cr_set_allocator()
    assert calls == []
