"""Launch modes of the reduction (one workgroup per tile, persistent work
queue, persistent inside a replayed hipGraph) and the autotuner: every mode
and every (policy, mode) pair gives the same bits."""
import numpy as np
import pytest

from paper_2602_24155_amd import crfrob as C
from tests.gpu_common import assert_item_matches_oracle, run_batch, workload_items

pytestmark = pytest.mark.gpu

MODES = [C.LAUNCH_PERSISTENT, C.LAUNCH_GRAPH]


@pytest.mark.parametrize("policy", [C.CR_POLICY_DEPTH_FIRST, C.CR_POLICY_P_CHUNK])
@pytest.mark.parametrize("launch", MODES)
def test_mixed_primes(launch, policy):
    """Several digit counts (one persistent launch and queue each) and, for
    p-chunk, several phases with combines between them."""
    items = workload_items("quintic_curves_mixed", range(6))
    res = run_batch(3, 5, items, launch=launch, policy=policy)
    assert res["stats"].engine == C.ENGINE_AUTO
    for i, (p, c) in enumerate(items):
        assert_item_matches_oracle(res, i, 3, 5, p, c)


def test_graph_replays_match_eager():
    """The cached graph is replayed with other eager work and synchronisations
    in between; every replay equals the eager result."""
    a = workload_items("quintic_curves_mixed", range(16, 20))
    b = workload_items("quintic_curves_mixed", range(20, 23))
    want_a = run_batch(3, 5, a)
    want_b = run_batch(3, 5, b)
    for rep in range(3):
        got = run_batch(3, 5, a, launch=C.LAUNCH_GRAPH)
        assert np.array_equal(got["scaled"], want_a["scaled"]) and got["lpoly"] == want_a["lpoly"], rep
        other = run_batch(3, 5, b)  # eager work between replays
        assert np.array_equal(other["scaled"], want_b["scaled"])
        got_b = run_batch(3, 5, b, launch=C.LAUNCH_GRAPH)
        assert np.array_equal(got_b["scaled"], want_b["scaled"]), rep


def test_full_size_launch_modes_agree():
    items = workload_items("quintic_curves_p31", range(256))
    base = run_batch(3, 5, items)
    for launch in MODES:
        for rep in range(2):
            res = run_batch(3, 5, items, launch=launch)
            assert np.array_equal(res["scaled"], base["scaled"]) and res["lpoly"] == base["lpoly"], (launch, rep)


def test_autotune_small_batch():
    items = workload_items("quintic_curves_p31", range(8))
    fam = C.family(3, 5)
    tu = C.cr_autotune(fam, [p for p, _ in items], [c for _, c in items], trials=1)
    ms = list(tu.ms)
    assert all(ms[pol * 3 + lm] > 0 for pol in range(3) for lm in range(3))
    assert tu.best_ms == ms[tu.best_policy * 3 + tu.best_launch] == min(x for x in ms if x > 0)
    res = run_batch(3, 5, items, policy=tu.best_policy, launch=tu.best_launch)
    base = run_batch(3, 5, items)
    assert np.array_equal(res["scaled"], base["scaled"])
