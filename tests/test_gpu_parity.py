"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Bar: bit-exact.  Every comparison is on integers: the scaled Frobenius
coordinates mod p^M, Phi' mod p^(column precision), column poles/precisions
and the integer L-polynomial.
"""
import numpy as np
import pytest

from oracle.diagonal import fermat_coeffs
from oracle.frobenius import frobenius
from oracle.lpoly import weil_root_check
from oracle.pointcount import count_projective
from oracle.poly import from_coeffs
from paper_2602_24155_amd import crfrob as C
from tests.gpu_common import assert_item_matches_oracle, run_batch, workload_items

pytestmark = pytest.mark.gpu


ENGINES = [C.ENGINE_AUTO, C.ENGINE_VALU, C.ENGINE_MFMA_LDS, C.ENGINE_MFMA_SINGLE]


@pytest.mark.parametrize("engine", ENGINES)
def test_quartic_curve_f7(engine):
    items = workload_items("quartic_curve_f7", [0])
    res = run_batch(3, 4, items, engine=engine)
    assert res["stats"].engine == engine
    assert_item_matches_oracle(res, 0, 3, 4, *items[0])


@pytest.mark.parametrize("engine", ENGINES)
def test_quintic_curves_mixed_primes(engine):
    items = workload_items("quintic_curves_mixed", range(6))
    res = run_batch(3, 5, items, engine=engine)
    assert res["stats"].engine == engine
    for i, (p, c) in enumerate(items):
        assert_item_matches_oracle(res, i, 3, 5, p, c)


def test_every_quintic_prime_both_engines():
    """One curve for each prime of the mixed workload (11..47): every digit base
    (B = 121, 169, then B = p) against the oracle, both kernels."""
    from tests.gpu_common import oracle_smooth
    from paper_2602_24155_amd import workload
    acc = oracle_smooth(3, 5)
    items = []
    for p in (11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47):
        rng = np.random.default_rng(p)
        while True:
            c = [int(x) for x in rng.integers(0, p, size=21)]
            if acc(p, c):
                items.append((p, c))
                break
    runs = [run_batch(3, 5, items, engine=e) for e in ENGINES]
    for e, res in zip(ENGINES, runs):
        assert res["stats"].engine == e
        for i, (p, c) in enumerate(items):
            assert_item_matches_oracle(res, i, 3, 5, p, c)


def test_quintic_curves_p31():
    items = workload_items("quintic_curves_p31", range(3))
    res = run_batch(3, 5, items)
    for i, (p, c) in enumerate(items):
        assert_item_matches_oracle(res, i, 3, 5, p, c)


@pytest.mark.parametrize("nv,d,p", [(3, 4, 7), (3, 4, 13), (3, 5, 11), (3, 5, 19), (3, 5, 41), (4, 4, 7),
                                    (4, 4, 13)])
def test_fermat(nv, d, p):
    c = fermat_coeffs(nv, d)
    res = run_batch(nv, d, [(p, c)])
    assert_item_matches_oracle(res, 0, nv, d, p, c)


def test_ragged_batch_and_bad_items():
    """Mixed batch: valid items of several primes around singular / invalid ones."""
    good = workload_items("quintic_curves_mixed", range(6, 9))
    items = [good[0], (31, [0] * 21), good[1], (11, [1] + [0] * 20), good[2]]
    fam = C.family(3, 5)
    res = C.cr_frobenius_batch(fam, [p for p, _ in items], [c for _, c in items], raise_on_error=False)
    assert res["status"] == C.CR_ESINGULAR
    assert list(res["item_status"]) == [0, C.CR_ESINGULAR, 0, C.CR_ESINGULAR, 0]
    for i in (0, 2, 4):
        assert_item_matches_oracle(res, i, 3, 5, *items[i])


def test_repeated_calls_identical():
    items = workload_items("quintic_curves_mixed", range(9, 11))
    a = run_batch(3, 5, items)
    b = run_batch(3, 5, items)
    assert np.array_equal(a["scaled"], b["scaled"]) and a["lpoly"] == b["lpoly"]


def test_empty_batch():
    res = C.cr_frobenius_batch(C.family(3, 5), [], np.zeros((0, 21), dtype=np.uint32))
    assert res["status"] == C.CR_OK


def test_full_size_headline_batch():
    """256 random quintic curves at p = 31 in one call (the benchmark launch):
    every item satisfies the Weil bound and the brute-force count #C(F_31);
    sampled items are compared with the oracle bit for bit."""
    items = workload_items("quintic_curves_p31", range(256))
    res = run_batch(3, 5, items)
    assert res["status"] == C.CR_OK
    for i, (p, c) in enumerate(items):
        a = res["lpoly"][i]
        assert len(a) == 13 and a[0] == 1 and a[12] == p ** 6
        assert weil_root_check(a, p, 1)
        if i % 16 == 0:
            assert count_projective(from_coeffs(3, 5, c), 3, p, 1) == p + 1 + a[1]
    for i in (0, 100, 255):
        assert_item_matches_oracle(res, i, 3, 5, *items[i])


def test_full_size_engines_agree():
    """The MFMA and VALU kernels give bit-identical results on the 256-curve batch."""
    items = workload_items("quintic_curves_p31", range(256))
    runs = [run_batch(3, 5, items, engine=e) for e in ENGINES]
    for e, res in zip(ENGINES, runs):
        assert res["stats"].engine == e
        assert np.array_equal(res["scaled"], runs[0]["scaled"])
        assert res["lpoly"] == runs[0]["lpoly"]


def test_release_regrow_and_invalid_items():
    """The device buffers (sub-batch arenas, the call's psi buffer) are freed by
    cr_release and grow again; items the setup rejects (p not prime, a
    coefficient not reduced mod p) sit beside valid ones, whose results
    are unchanged."""
    small = workload_items("quintic_curves_mixed", range(3))
    a = run_batch(3, 5, small)
    C.cr_release()
    big = workload_items("quintic_curves_mixed", range(40))
    b = run_batch(3, 5, big)
    for i in range(3):
        assert np.array_equal(a["scaled"][i], b["scaled"][i]) and a["lpoly"][i] == b["lpoly"][i]
    bad = [(9, [1] * 21), (small[0][0], [small[0][0]] + [0] * 20)]
    items = [small[0], bad[0], small[1], bad[1], small[2]]
    res = C.cr_frobenius_batch(C.family(3, 5), [p for p, _ in items], [c for _, c in items], raise_on_error=False)
    st = list(res["item_status"])
    assert st[0] == st[2] == st[4] == C.CR_OK and st[1] != C.CR_OK and st[3] != C.CR_OK
    for i, j in ((0, 0), (2, 1), (4, 2)):
        assert np.array_equal(res["scaled"][i], a["scaled"][j]) and res["lpoly"][i] == a["lpoly"][j]


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("policy", [C.CR_POLICY_DEPTH_FIRST, C.CR_POLICY_P_CHUNK, C.CR_POLICY_VAR_BY_VAR])
def test_s_mask_subsets(engine, policy):
    """S a proper subset of the variables (Definition 3.1; Proposition 3.3 in
    the x^S form): the device reduction with cr_family.s_mask against the
    oracle run with the same S, bit for bit, for the quartic curve over F_7
    and a quintic curve over F_37, several S each."""
    from oracle.cohomology import is_s_smooth
    if engine == C.ENGINE_MFMA_LDS and policy != C.CR_POLICY_DEPTH_FIRST:
        pytest.skip("the LDS-gather kernel runs the depth-first policy only")
    cases = [("quartic_curve_f7", 3, 4, 0, [[2], [0], [1, 2]]), ("quintic_curves_mixed", 3, 5, 1, [[0], [1, 2]])]
    for name, nv, d, j, subsets in cases:
        p, c = workload_items(name, [j])[0]
        fp = {e: v % p for e, v in from_coeffs(nv, d, c).items() if v % p}
        for S in subsets:
            assert is_s_smooth(fp, nv, d, p, S)
            mask = sum(1 << i for i in S)
            res = run_batch(nv, d, [(p, c)], s_mask=mask, engine=engine, policy=policy)
            o = frobenius(nv, d, p, c, S=S)
            print("s_mask case", name, p, S, "engine", res["stats"].engine, flush=True)
            assert_item_matches_oracle(res, 0, nv, d, p, c, oracle=o)


@pytest.mark.parametrize("engine", [C.ENGINE_AUTO, C.ENGINE_VALU])
def test_single_entry_and_precision_overrides(engine):
    """cr_frobenius (one hypersurface) with the working precision M and the
    per-pole series orders N_m overridden (Section 2.5, Proposition 2.1),
    against the oracle run with the same overrides, bit for bit."""
    for name, nv, d in (("quartic_curve_f7", 3, 4), ("quintic_curves_p31", 3, 5)):
        p, c = workload_items(name, [0])[0]
        r, N, M = C.cr_precision(C.family(nv, d), p)
        cases = [({}, {}), ({"M": M + 2}, {"M": M + 2}), ({"n_series_m": [N + 1, N]}, {"N": {1: N + 1, 2: N}})]
        for kw, okw in cases:
            print("precision case", name, kw, flush=True)
            one = C.cr_frobenius(C.family(nv, d, engine=engine, **kw), p, c)
            res = {k: [v] for k, v in one.items() if k in ("frob", "scaled", "col_pole", "col_prec", "lpoly")}
            res["item_status"] = [one["status"]]
            o = frobenius(nv, d, p, c, **okw)
            assert_item_matches_oracle(res, 0, nv, d, p, c, oracle=o)


def test_full_mixed_prime_batch():
    """The whole 256-curve mixed-prime workload (p uniform over 11..47) in one
    call: every item satisfies the Weil bound and the brute-force #C(F_p), and
    the first curve of each prime is compared with the oracle bit for bit."""
    items = workload_items("quintic_curves_mixed", range(256))
    res = run_batch(3, 5, items, launch=C.LAUNCH_PERSISTENT)
    assert res["status"] == C.CR_OK
    first = {}
    for i, (p, c) in enumerate(items):
        a = res["lpoly"][i]
        assert len(a) == 13 and a[0] == 1 and a[12] == p ** 6
        assert weil_root_check(a, p, 1)
        assert count_projective(from_coeffs(3, 5, c), 3, p, 1) == p + 1 + a[1]
        first.setdefault(p, i)
    assert sorted(first) == [11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47]
    for p, i in sorted(first.items()):
        print("mixed batch: oracle check of item %d (p = %d)" % (i, p), flush=True)
        assert_item_matches_oracle(res, i, 3, 5, *items[i])
