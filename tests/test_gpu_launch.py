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


def test_autotune_small_batch(tmp_path):
    """Stage 1 times every (policy, launch) pair, stage 2 the kernel shapes
    (engine x persistent grid) of the best pair; the best configuration gives
    the same bits; a cache file returns the same choice without timing."""
    items = workload_items("quintic_curves_p31", range(8))
    primes, coeffs = [p for p, _ in items], [c for _, c in items]
    fam = C.family(3, 5)
    cache = str(tmp_path / "tune.txt")
    C.cr_autotune_cache(cache)
    try:
        tu = C.cr_autotune(fam, primes, coeffs, trials=1)
        assert tu.from_cache == 0
        ms = list(tu.ms)
        assert all(ms[pol * 3 + lm] > 0 for pol in range(3) for lm in range(3))
        shapes = list(tu.shape_ms)
        # plane quintics: auto (tile pairs), single tiles, LDS gather and VALU run; the quad kernel does not
        assert shapes[0] > 0 and shapes[2] > 0 and shapes[7] > 0 and shapes[5] < 0 and shapes[6] < 0
        assert tu.best_ms == min(x for x in ms + shapes if x > 0)
        res = run_batch(3, 5, items, policy=tu.best_policy, launch=tu.best_launch, engine=tu.best_engine,
                        grid=tu.best_grid)
        base = run_batch(3, 5, items)
        assert np.array_equal(res["scaled"], base["scaled"]) and res["lpoly"] == base["lpoly"]
        again = C.cr_autotune(fam, primes, coeffs, trials=1)
        assert again.from_cache == 1
        assert (again.best_policy, again.best_launch, again.best_engine, again.best_grid) == \
            (tu.best_policy, tu.best_launch, tu.best_engine, tu.best_grid)
        assert open(cache).read().count("\n") == 1
    finally:
        C.cr_autotune_cache(None)


@pytest.mark.parametrize("grid", [1, 2])
def test_persistent_grid_sizes(grid):
    items = workload_items("quintic_curves_mixed", range(6))
    base = run_batch(3, 5, items)
    for engine in (C.ENGINE_AUTO, C.ENGINE_MFMA_SINGLE):
        res = run_batch(3, 5, items, launch=C.LAUNCH_PERSISTENT, grid=grid, engine=engine)
        assert res["stats"].engine == engine
        assert np.array_equal(res["scaled"], base["scaled"]) and res["lpoly"] == base["lpoly"]
