"""GPU parity of the combining policies (Section 4): every policy must give the
oracle's bits.  The scaled Frobenius coordinates mod p^M are the same for
every valid reduction path (each step is an exact identity in cohomology and
coordinates in the basis are unique), so the depth-first oracle is the
reference for all of them."""
import numpy as np
import pytest

from oracle.diagonal import fermat_coeffs
from paper_2602_24155_amd import crfrob as C
from tests.gpu_common import assert_item_matches_oracle, run_batch, workload_items

pytestmark = pytest.mark.gpu

COMBINING = [C.CR_POLICY_P_CHUNK, C.CR_POLICY_VAR_BY_VAR]
ENGINES = [C.ENGINE_AUTO, C.ENGINE_VALU, C.ENGINE_MFMA_SINGLE]


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("policy", COMBINING)
def test_quartic_curve_f7(policy, engine):
    items = workload_items("quartic_curve_f7", [0])
    res = run_batch(3, 4, items, policy=policy, engine=engine)
    assert res["stats"].policy == policy and res["stats"].engine == engine
    assert_item_matches_oracle(res, 0, 3, 4, *items[0])


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("policy", COMBINING)
def test_quintic_curves_mixed_primes(policy, engine):
    items = workload_items("quintic_curves_mixed", range(6))
    res = run_batch(3, 5, items, policy=policy, engine=engine)
    st = res["stats"]
    assert st.policy == policy and st.engine == engine and st.phases > 1
    assert st.merged_terms > 0
    for i, (p, c) in enumerate(items):
        assert_item_matches_oracle(res, i, 3, 5, p, c)


@pytest.mark.parametrize("policy", COMBINING)
def test_fermat_k3(policy):
    c = fermat_coeffs(4, 4)
    res = run_batch(4, 4, [(7, c)], policy=policy)
    assert res["stats"].policy == policy
    assert_item_matches_oracle(res, 0, 4, 4, 7, c)


def test_full_size_policies_agree():
    """256 curves at p = 31: p-chunk and var-by-var give the depth-first bits
    with fewer column steps."""
    items = workload_items("quintic_curves_p31", range(256))
    base = run_batch(3, 5, items)
    for pol in COMBINING:
        res = run_batch(3, 5, items, policy=pol)
        assert res["status"] == C.CR_OK and res["stats"].policy == pol
        assert np.array_equal(res["scaled"], base["scaled"])
        assert res["lpoly"] == base["lpoly"]
        assert res["stats"].column_steps < base["stats"].column_steps


@pytest.mark.parametrize("policy", [C.CR_POLICY_DEPTH_FIRST] + COMBINING)
def test_batch_counters_match_the_host_game(policy):
    """The counters of a batch call (the depth-first chunk count is taken while
    the device runs) equal the sums of cr_policy_cost over its items."""
    items = workload_items("quintic_curves_mixed", range(40))
    res = run_batch(3, 5, items, policy=policy)
    fam = C.family(3, 5, policy=policy)
    want = {k: 0 for k in ("column_steps", "chunks", "vectors", "merged_terms")}
    for p, c in items:
        cost = C.cr_policy_cost(fam, p, c)
        for k in want:
            want[k] += getattr(cost, k)
    for k, v in want.items():
        assert getattr(res["stats"], k) == v, k
