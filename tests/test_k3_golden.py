"""Random quartic K3 surfaces over F_7, F_11 and F_13: stored oracle results.

tests/golden/k3_golden.json is written by tests/golden/make_k3_golden.py,
which calls only oracle/ (about a minute and a half per surface; four per
prime, the first of each prime in workload order).  On the CPU the stored
L-polynomials are checked against facts independent of the oracle (Weil
bounds and the functional equation, #X(F_p) by brute force, the inputs being
the workload's); on the GPU the library is compared with them bit for bit,
under every policy.
"""
import json
import os

import numpy as np
import pytest

from oracle.lpoly import point_counts_from_lpoly, weil_root_check_squarefree
from oracle.poly import from_coeffs
from oracle.pointcount import count_projective
from paper_2602_24155_amd import crfrob as C
from paper_2602_24155_amd import workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "k3_golden.json")


def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)["items"]


def test_golden_inputs_are_the_workload_items():
    for it in golden():
        p, c = workload.first_accepted("quartic_k3_mixed", it["j"], lambda p_, c_: True)
        assert p == it["p"]
        # the stored candidate is one of the stream's candidates (the first smooth one)
        _p, gen = workload.stream("quartic_k3_mixed", it["j"])
        assert any(next(gen) == it["coeffs"] for _ in range(64))
    ps = [it["p"] for it in golden()]
    assert all(ps.count(p) >= 4 for p in (7, 11, 13))


def test_golden_lpolys_satisfy_weil_and_point_counts():
    for it in golden():
        p = it["p"]
        a = [int(x) for x in it["lpoly"]]
        assert len(a) == 22 and a[0] == 1 and abs(a[21]) == p ** 21
        assert weil_root_check_squarefree(a, p, 2)
        f = {e: v % p for e, v in from_coeffs(4, 4, it["coeffs"]).items() if v % p}
        assert point_counts_from_lpoly(a, p, 3, 1) == [count_projective(f, 4, p, 1)]


def test_golden_lpolys_match_counts_over_f_p2():
    """#X(F_{p^2}) by brute force (per-line root counts over F_{p^2}) fixes the
    power sum s_2 of the Frobenius eigenvalues, a second independent
    combination of the stored coefficients (a_1^2 - 2 a_2).  One surface per
    prime (the count over F_{13^2} takes about 20 s)."""
    seen = set()
    for it in golden():
        if it["p"] in seen:
            continue
        seen.add(it["p"])
        p = it["p"]
        a = [int(x) for x in it["lpoly"]]
        f = {e: v % p for e, v in from_coeffs(4, 4, it["coeffs"]).items() if v % p}
        assert point_counts_from_lpoly(a, p, 3, 2) == [count_projective(f, 4, p, k) for k in (1, 2)]


@pytest.mark.gpu
@pytest.mark.parametrize("policy", [C.CR_POLICY_DEPTH_FIRST, C.CR_POLICY_P_CHUNK, C.CR_POLICY_VAR_BY_VAR])
def test_gpu_matches_golden(policy):
    items = golden()
    fam = C.family(4, 4, policy=policy)
    res = C.cr_frobenius_batch(fam, [it["p"] for it in items], [it["coeffs"] for it in items])
    assert res["stats"].policy == policy
    for i, it in enumerate(items):
        assert res["item_status"][i] == 0
        assert [[int(x) for x in row] for row in res["scaled"][i]] == [[int(x) for x in row] for row in it["scaled"]]
        assert [int(x) for x in res["col_pole"][i]] == it["col_pole"]
        assert [int(x) for x in res["col_prec"][i]] == it["col_prec"]
        prec = it["col_prec"]
        want = [[int(x) % it["p"] ** prec[c_] for c_, x in enumerate(row)] for row in it["phi_prime"]]
        assert [[int(x) for x in row] for row in res["frob"][i]] == want
        assert res["lpoly"][i] == [int(x) for x in it["lpoly"]]
