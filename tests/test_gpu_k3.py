"""GPU parity of the quartic K3 surfaces (four variables, s = 220, 21-dimensional
primitive H^2): the int8-digit MFMA quad kernel and the 64-bit VALU kernel
against the oracle's stored results (tests/golden/k3_golden.json, written by
make_k3_golden.py from oracle/ only), under every plain policy and launch
mode, and the whole 64-surface workload in one call checked item by item
against the Weil bound, the functional equation and #X(F_p)."""
import json
import os

import numpy as np
import pytest

from oracle.diagonal import fermat_coeffs
from oracle.lpoly import weil_root_check_squarefree
from oracle.pointcount import count_projective
from oracle.poly import from_coeffs
from paper_2602_24155_amd import crfrob as C
from paper_2602_24155_amd import workload
from tests.gpu_common import assert_item_matches_oracle, run_batch

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "k3_golden.json")))["items"]
POLICIES = [C.CR_POLICY_DEPTH_FIRST, C.CR_POLICY_P_CHUNK, C.CR_POLICY_VAR_BY_VAR]


def _assert_golden(res, i, g):
    assert res["item_status"][i] == 0
    assert [[int(x) for x in row] for row in res["scaled"][i]] == [[int(x) for x in row] for row in g["scaled"]]
    assert [int(x) for x in res["col_pole"][i]] == g["col_pole"]
    assert [int(x) for x in res["col_prec"][i]] == g["col_prec"]
    b = len(g["col_pole"])
    for r in range(b):
        for c in range(b):
            assert int(res["frob"][i][r][c]) == int(g["phi_prime"][r][c]) % g["p"] ** g["col_prec"][c]
    assert res["lpoly"][i] == [int(a) for a in g["lpoly"]]


@pytest.mark.parametrize("policy", POLICIES)
def test_goldens_quad_kernel(policy):
    """The twelve stored random K3 surfaces (four each at p = 7, 11, 13: digit counts 9, 7, 7)
    in one call on the quad kernel, bit for bit."""
    res = run_batch(4, 4, [(g["p"], g["coeffs"]) for g in GOLD], policy=policy)
    assert res["stats"].engine == C.ENGINE_QUAD and res["stats"].policy == policy
    for i, g in enumerate(GOLD):
        print("golden j=%d p=%d policy %d" % (g["j"], g["p"], policy), flush=True)
        _assert_golden(res, i, g)


@pytest.mark.parametrize("launch", [C.LAUNCH_PERSISTENT, C.LAUNCH_GRAPH])
def test_goldens_quad_launch_modes(launch):
    res = run_batch(4, 4, [(g["p"], g["coeffs"]) for g in GOLD], policy=C.CR_POLICY_P_CHUNK, launch=launch)
    assert res["stats"].engine == C.ENGINE_QUAD
    for i, g in enumerate(GOLD):
        _assert_golden(res, i, g)


def test_goldens_valu_kernel():
    res = run_batch(4, 4, [(g["p"], g["coeffs"]) for g in GOLD], policy=C.CR_POLICY_P_CHUNK, engine=C.ENGINE_VALU)
    assert res["stats"].engine == C.ENGINE_VALU
    for i, g in enumerate(GOLD):
        _assert_golden(res, i, g)


@pytest.mark.parametrize("p", [7, 11, 13])
def test_fermat_k3_quad_kernel(p):
    c = fermat_coeffs(4, 4)
    res = run_batch(4, 4, [(p, c)], policy=C.CR_POLICY_P_CHUNK)
    assert res["stats"].engine == C.ENGINE_QUAD
    assert_item_matches_oracle(res, 0, 4, 4, p, c)


def test_full_k3_workload():
    """The 64 random K3 surfaces of the workload (p in {7, 11, 13}) in one call:
    every Q(T) has a_0 = 1, satisfies the functional equation with sign +-1 and
    the Weil bound, and its a_1 matches the brute-force #X(F_p); the stored
    goldens among them are bit-exact."""
    w = workload.WORKLOADS["quartic_k3_mixed"]
    fam = C.family(4, 4)
    items = [workload.first_accepted(w, j, lambda p, c: C.cr_check_smooth(fam, p, c)) for j in range(w.count)]
    res = run_batch(4, 4, items, policy=C.CR_POLICY_P_CHUNK, launch=C.LAUNCH_PERSISTENT)
    assert res["status"] == C.CR_OK and res["stats"].engine == C.ENGINE_QUAD
    print("64 K3: reduce %.1f ms, %d column steps" % (res["stats"].reduce_ms, res["stats"].column_steps), flush=True)
    for i, (p, c) in enumerate(items):
        a = res["lpoly"][i]
        assert len(a) == 22 and a[0] == 1
        eps = a[21] // p ** 21
        assert eps in (1, -1) and a[21] == eps * p ** 21
        for k in range(11):  # functional equation, weight 2
            assert a[21 - k] == eps * p ** (21 - 2 * k) * a[k]
        assert weil_root_check_squarefree(a, p, 2), (i, p, a)
        # #X(F_p) = 1 + p + p^2 + sum of the roots alpha_j = 1 + p + p^2 - a_1
        assert count_projective(from_coeffs(4, 4, c), 4, p, 1) == 1 + p + p * p - a[1]
    for g in GOLD:
        _assert_golden(res, g["j"], g)
    # Artin-Mazur heights (Section 6.3) of the batch: library against the oracle's definitions
    from collections import Counter
    from oracle.newton import invariants
    heights = Counter()
    for i, (p, c) in enumerate(items):
        lib = C.cr_newton_polygon(4, 4, p, C.lpoly_words(res["lpoly"][i]))
        inv = invariants(res["lpoly"][i], p, 3, {1: 1, 2: 19, 3: 1})
        h = inv["height"]
        assert lib.height == (0 if h == float("inf") else int(h))
        assert (lib.domino_num, lib.domino_den) == (inv["domino"].numerator, inv["domino"].denominator)
        heights[(p, lib.height)] += 1
    print("heights (p, h): count", sorted(heights.items()), flush=True)
