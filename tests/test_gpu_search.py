"""Sparse hypersurfaces and the Newton-polygon search of Section 6.1 on the GPU.

* Six-term quartic surfaces (the Fermat quartic plus two random monomials,
  the shape of Table 2 and of Method 2's deformations) through the quad
  kernel, bit for bit against the oracle.
* Method 2 around the Fermat quartic over F_7 (supersingular, p = 3 mod 4)
  and Method 1 over F_7: every candidate's Newton invariants from the
  library agree with the oracle's definitions on the same Q(T), heights lie
  in {1..10} or are infinite (Section 6.3), and the search keeps exactly the
  candidates its predicate accepts.
"""
from collections import Counter

import pytest

from oracle.frobenius import frobenius
from oracle.newton import invariants as oracle_invariants
from paper_2602_24155_amd import crfrob as C
from paper_2602_24155_amd import search, workload
from tests.gpu_common import assert_item_matches_oracle

pytestmark = pytest.mark.gpu

K3_HODGE = {1: 1, 2: 19, 3: 1}


def test_sparse_k3_against_oracle():
    w = workload.WORKLOADS["sparse_k3_mixed"]
    fam = C.family(4, 4)
    items = [workload.first_accepted(w, j, lambda p, c: C.cr_check_smooth(fam, p, c)) for j in range(3)]
    oracles = [frobenius(4, 4, p, c) for p, c in items]
    for policy in (C.CR_POLICY_DEPTH_FIRST, C.CR_POLICY_P_CHUNK):
        res = C.cr_frobenius_batch(C.family(4, 4, policy=policy), [p for p, _ in items], [c for _, c in items])
        assert res["stats"].engine == C.ENGINE_QUAD
        for i, (p, c) in enumerate(items):
            print("sparse K3 j=%d p=%d policy %d" % (i, p, policy), flush=True)
            assert sum(1 for x in c if x) == 6
            assert_item_matches_oracle(res, i, 4, 4, p, c, oracle=oracles[i])


@pytest.mark.parametrize("method", [1, 2])
def test_newton_search_k3_p7(method):
    found, seen = search.search(4, 4, 7, lambda inv: inv["height"] is not None and inv["height"] >= 2,
                                count=32, seed=5, method=method, extra_terms=1)
    assert len(seen) == 32
    hist = Counter(inv["height"] for inv in seen)
    print("method %d heights over F_7:" % method, sorted(hist.items(), key=lambda kv: kv[0]), flush=True)
    for inv in seen:
        h = inv["height"]
        assert h == float("inf") or h in range(1, 11)
    assert len(found) == sum(1 for inv in seen if inv["height"] >= 2)
    for f in found:
        o = oracle_invariants(f["lpoly"], 7, 3, K3_HODGE)
        assert o["height"] == f["invariants"]["height"] and o["height"] >= 2
        assert o["domino"] == f["invariants"]["domino"]
        assert o["supersingular"] == f["invariants"]["supersingular"]
