"""Reduction policies on the CPU: the library's host planner (cr_policy_cost)
against the oracle's game of Section 3.4 (oracle/policy.py), and the oracle's
game against facts that do not depend on it."""
import pytest

from oracle import policy as OP
from paper_2602_24155_amd import crfrob as C
from tests.gpu_common import workload_items

POLICIES = [("depth_first", C.CR_POLICY_DEPTH_FIRST), ("p_chunk", C.CR_POLICY_P_CHUNK),
            ("var_by_var", C.CR_POLICY_VAR_BY_VAR)]
FIELDS = ["column_steps", "chunks", "vectors", "merged_terms", "combined_groups", "phases"]


def test_greedy_direction_by_hand():
    # Algorithm 3, d = 5, S = all: units on x0 and x2, then x0, x2, x0
    assert OP.greedy_direction((10, 0, 3), 5, [0, 1, 2]) == [3, 0, 2]
    # every variable used once, then round robin from x0
    assert OP.greedy_direction((4, 4, 4), 5, [0, 1, 2]) == [2, 2, 1]
    # S = {2}: the unit loop only looks at x2
    assert OP.greedy_direction((1, 9, 0), 4, [2]) == [1, 3, 0]
    # |u| < d: no direction
    assert OP.greedy_direction((1, 1, 1), 5, [0, 1, 2]) is None


def test_tweak_by_hand():
    # Algorithm 1 removes k units from the front
    assert OP.tweak((3, 5, 2), 6) == ((0, 2, 2), (3, 3, 0))
    assert OP.tweak((0, 0, 9), 4) == ((0, 0, 5), (0, 0, 4))


@pytest.fixture(scope="module")
def cases():
    out = [(3, 4) + workload_items("quartic_curve_f7", [0])[0]]
    out += [(3, 5) + it for it in workload_items("quintic_curves_mixed", range(3))]
    out += [(3, 5) + workload_items("quintic_curves_p31", [0])[0]]
    return [(nv, d, p, c, OP.start_terms(nv, d, p, c)) for nv, d, p, c in out]


def test_game_facts(cases):
    """Facts about the game that do not come from the simulation itself: depth
    first reduces every term one pole order per step (sum of P - n column steps,
    one vector per start term, no combining); p-chunk has one phase per pole
    level (every start pole is a multiple of p); combining never adds work."""
    for nv, d, p, c, starts in cases:
        n = nv - 1
        df = OP.play(nv, d, p, starts, "depth_first")
        assert df["column_steps"] == sum(pole - n for _u, pole, _c in starts)
        assert df["vectors"] == len(starts) and df.get("merged_terms", 0) == 0
        assert all(pole % p == 0 for _u, pole, _c in starts)
        pc = OP.play(nv, d, p, starts, "p_chunk")
        assert pc["phases"] == len({pole for _u, pole, _c in starts})
        vv = OP.play(nv, d, p, starts, "var_by_var")
        assert pc["column_steps"] <= df["column_steps"] and vv["column_steps"] <= df["column_steps"]
        assert vv["phases"] <= nv + 1


def test_p_chunk_saves_work_at_p31(cases):
    nv, d, p, c, starts = cases[-1]
    assert p == 31
    df = OP.play(nv, d, p, starts, "depth_first")
    pc = OP.play(nv, d, p, starts, "p_chunk")
    assert pc["merged_terms"] > 0 and pc["column_steps"] < 0.9 * df["column_steps"]


@pytest.mark.parametrize("name,pol", POLICIES)
def test_planner_matches_oracle_game(cases, name, pol):
    for nv, d, p, c, starts in cases:
        fam = C.family(nv, d, policy=pol)
        st = C.cr_policy_cost(fam, p, c)
        want = OP.play(nv, d, p, starts, name)
        got = {k: getattr(st, k) for k in FIELDS}
        assert st.start_blocks == len(starts)
        assert got == {k: want.get(k, 0) for k in FIELDS}, (name, p)


def test_learned_policy_needs_model():
    nv, d = 3, 4
    p, c = workload_items("quartic_curve_f7", [0])[0]
    with pytest.raises(C.CrError) as e:
        C.cr_policy_cost(C.family(nv, d, policy=C.CR_POLICY_LEARNED), p, c)
    assert e.value.status == C.CR_EINVAL
