"""A random cubic threefold over F_7 with S = {x_4} (Definition 3.1; Section 6.5).

tests/golden/cubic_threefold_golden.json is written by
tests/golden/make_cubic_threefold_golden.py, which calls only oracle/ (about
ten minutes).  The stored L-polynomial is checked against facts independent
of the oracle: the functional equation and the Weil bound for weight 3, and
#X(F_7), #X(F_49) by brute force (the first two power sums of the Frobenius
eigenvalues).  Its Newton invariants (Section 6.5: p-rank = length of the
slope-1 segment) agree between the library's host routine and the oracle.

On the GPU the threefold kernel (int8-digit MFMA over the 1815 x 1001 right
inverse of J_S) reproduces the stored result bit for bit; cubic fourfolds,
which no kernel covers, are refused with CR_EINVAL.
"""
import json
import os
from fractions import Fraction

import pytest

from oracle.lpoly import point_counts_from_lpoly, weil_root_check_squarefree
from oracle.newton import invariants
from oracle.pointcount import count_projective
from oracle.poly import from_coeffs
from paper_2602_24155_amd import crfrob as C
from paper_2602_24155_amd import workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cubic_threefold_golden.json")
FACTS = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")


def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)["items"][0]


def test_golden_input_is_the_workload_item():
    g = golden()
    p, gen = workload.stream("cubic_threefold_f7", g["j"])
    assert p == g["p"] == 7
    assert any(next(gen) == g["coeffs"] for _ in range(64))


def test_golden_lpoly_functional_equation_and_weil():
    g = golden()
    p = g["p"]
    a = [int(x) for x in g["lpoly"]]
    facts = [f for f in json.load(open(FACTS))["hodge_numbers"] if f["family"] == "cubic threefold"][0]
    b = facts["primitive_b"]
    assert len(a) == b + 1 and a[0] == 1
    # weight 3: a_{b-j} = sign * p^{3(b/2 - j)} a_j, sign = +1 or -1
    sign = a[b] // p ** (3 * b // 2)
    assert sign in (1, -1) and a[b] == sign * p ** (3 * b // 2)
    for j in range(b + 1):
        assert a[b - j] * p ** (3 * j) == sign * p ** (3 * b // 2) * a[j]
    assert weil_root_check_squarefree(a, p, 3)


def test_golden_lpoly_matches_point_counts():
    g = golden()
    p = g["p"]
    a = [int(x) for x in g["lpoly"]]
    f = {e: v % p for e, v in from_coeffs(5, 3, g["coeffs"]).items() if v % p}
    assert point_counts_from_lpoly(a, p, 4, 2) == [count_projective(f, 5, p, k) for k in (1, 2)]


def _hodge():
    h = [f for f in json.load(open(FACTS))["hodge_numbers"] if f["family"] == "cubic threefold"][0]["h"]
    # basis elements of pole order m carry Hodge slope n - m = 4 - m: h^{3,0} at m = 1, ..., h^{0,3} at m = 4
    return {m: h[m - 1] for m in range(1, 5)}


def test_newton_invariants_library_matches_oracle():
    g = golden()
    p = g["p"]
    a = [int(x) for x in g["lpoly"]]
    inv = invariants(a, p, 4, _hodge())
    # all slopes lie in [1, 2] (Mazur: Newton above Hodge, h^{3,0} = 0), symmetric about 3/2
    assert all(Fraction(1) <= s <= Fraction(2) for s, _ in inv["slopes"])
    assert sum(s * ln for s, ln in inv["slopes"]) == Fraction(3 * 10, 2)
    assert inv["height"] is None and inv["domino"] is None
    lib = C.cr_newton_polygon(5, 3, p, C.lpoly_words(a))
    slopes = [(Fraction(r, ln), ln) for ln, r in zip(lib.seg_len[:lib.nseg], lib.seg_rise[:lib.nseg])]
    assert slopes == inv["slopes"]
    assert lib.p_rank == inv["p_rank"]
    assert bool(lib.ordinary) == inv["ordinary"] and bool(lib.supersingular) == inv["supersingular"]
    assert lib.height == -1 and (lib.domino_num, lib.domino_den) == (-1, 1)


@pytest.mark.gpu
def test_gpu_threefold_kernel_matches_golden():
    """The threefold kernel (engine 5, int8-digit MFMA, 57 row tiles x 32
    K-blocks) against the oracle's stored result, bit for bit: the scaled
    matrix mod p^M, Phi' mod p^(column precision), column poles and
    precisions, and Q(T)."""
    g = golden()
    for policy in (C.CR_POLICY_DEPTH_FIRST, C.CR_POLICY_P_CHUNK):
        fam = C.family(5, 3, s_mask=1 << 4, policy=policy)
        res = C.cr_frobenius_batch(fam, [g["p"]], [g["coeffs"]])
        assert res["stats"].engine == C.ENGINE_WIDE and res["stats"].policy == policy
        assert [[int(x) for x in row] for row in res["scaled"][0]] == [[int(x) for x in row] for row in g["scaled"]]
        assert [int(x) for x in res["col_pole"][0]] == g["col_pole"]
        assert [int(x) for x in res["col_prec"][0]] == g["col_prec"]
        prec = g["col_prec"]
        want = [[int(x) % g["p"] ** prec[c] for c, x in enumerate(row)] for row in g["phi_prime"]]
        assert [[int(x) for x in row] for row in res["frob"][0]] == want
        assert res["lpoly"][0] == [int(x) for x in g["lpoly"]]


@pytest.mark.gpu
def test_gpu_threefold_batch_properties():
    """A batch of random cubic threefolds over F_7 and F_11 (the second prime
    of Section 5.3's example) with the golden threefold among them: every
    Q(T) satisfies the functional equation and the Weil bound in weight 3
    and gives #X(F_p) by brute force; the golden item is bit-exact."""
    fam = C.family(5, 3, s_mask=1 << 4)
    items = [workload.first_accepted("cubic_threefolds_mixed", j, lambda p, c: C.cr_check_smooth(fam, p, c))
             for j in range(6)]
    g = golden()
    items.insert(3, (g["p"], g["coeffs"]))
    assert {p for p, _ in items} == {7, 11}
    res = C.cr_frobenius_batch(fam, [p for p, _ in items], [c for _, c in items])
    assert res["stats"].engine == C.ENGINE_WIDE
    for i, (p, c) in enumerate(items):
        assert res["item_status"][i] == C.CR_OK
        a = res["lpoly"][i]
        assert len(a) == 11 and a[0] == 1 and abs(a[10]) == p ** 15
        assert weil_root_check_squarefree(a, p, 3)
        f = {e: v % p for e, v in from_coeffs(5, 3, c).items() if v % p}
        assert point_counts_from_lpoly(a, p, 4, 1) == [count_projective(f, 5, p, 1)]
    assert [[int(x) for x in row] for row in res["scaled"][3]] == [[int(x) for x in row] for row in g["scaled"]]
    assert res["lpoly"][3] == [int(x) for x in g["lpoly"]]


@pytest.mark.gpu
def test_gpu_refuses_family_without_device_path():
    """Cubic fourfolds (six variables, S = {x_5}): psi has 80 million entries
    and no MFMA kernel covers the family, so the call is refused before any
    setup (the coefficients are not even looked at)."""
    fam = C.family(6, 3, s_mask=1 << 5)
    nco, _s, _b = C.cr_query_dims(6, 3)
    with pytest.raises(C.CrError, match="no device path") as e:
        C.cr_frobenius_batch(fam, [7], [[1] * nco])
    assert e.value.status == C.CR_EINVAL


@pytest.mark.gpu
def test_gpu_rejects_a_threefold_that_is_not_s_smooth():
    """The first candidate of the workload's hypersurface 17 (over F_11) is not
    S-smooth for S = {x_4} (the host check says so): in a batch with the stored
    golden it gets CR_ENOT_S_SMOOTH from the device elimination of J_S, and
    the golden item's bits are unchanged."""
    fam = C.family(5, 3, s_mask=1 << 4)
    p, gen = workload.stream("cubic_threefolds_mixed", 17)
    bad = next(gen)
    assert p == 11 and not C.cr_check_smooth(fam, p, bad)
    g = golden()
    res = C.cr_frobenius_batch(fam, [g["p"], p], [g["coeffs"], bad], raise_on_error=False)
    assert list(res["item_status"]) == [C.CR_OK, C.CR_ENOT_S_SMOOTH]
    assert [[int(x) for x in row] for row in res["scaled"][0]] == [[int(x) for x in row] for row in g["scaled"]]
    assert res["lpoly"][0] == [int(x) for x in g["lpoly"]]
