"""cr_frobenius_batch_noalloc (every device buffer in the library's static
workspace) against cr_frobenius_batch: the same bits on two calls in a row,
the second with a smaller batch, under the combining and the depth-first
policy; the rejections the header documents."""
import numpy as np
import pytest

from paper_2602_24155_amd import crfrob as C
from paper_2602_24155_amd import workload

pytestmark = pytest.mark.gpu


def _items(name, js):
    w = workload.WORKLOADS[name]
    fam = C.family(w.nvars, w.degree)
    return [workload.first_accepted(w, j, lambda p, c: C.cr_check_smooth(fam, p, c)) for j in js]


def _same(a, b):
    assert a["status"] == b["status"] == 0
    assert np.array_equal(a["item_status"], b["item_status"])
    for k in ("frob", "scaled", "col_pole", "col_prec"):
        assert np.array_equal(a[k], b[k]), k
    assert a["lpoly"] == b["lpoly"]


@pytest.mark.parametrize("policy,launch", [(C.CR_POLICY_P_CHUNK, C.LAUNCH_PERSISTENT),
                                           (C.CR_POLICY_DEPTH_FIRST, C.LAUNCH_GRID)])
def test_noalloc_matches_batch_on_two_calls(policy, launch):
    big = _items("quintic_curves_mixed", range(40))  # more than one sub-batch: both workspace slices
    small = _items("quintic_curves_mixed", range(40, 47))
    for items in (big, small):
        fam = C.family(3, 5, policy=policy, launch=launch)
        primes = [p for p, _ in items]
        coeffs = [c for _, c in items]
        want = C.cr_frobenius_batch(fam, primes, coeffs)
        got = C.cr_frobenius_batch(fam, primes, coeffs, noalloc=True)
        _same(got, want)
        assert got["stats"].column_steps == want["stats"].column_steps


def test_noalloc_quartic_curve_and_again_after_a_larger_call():
    """A one-item call right after a larger one (stale workspace contents)."""
    items = _items("quartic_curve_f7", [0])
    fam = C.family(3, 4)
    want = C.cr_frobenius_batch(fam, [items[0][0]], [items[0][1]])
    got = C.cr_frobenius_batch(fam, [items[0][0]], [items[0][1]], noalloc=True)
    _same(got, want)


def test_noalloc_rejections():
    items = _items("quintic_curves_mixed", range(2))
    primes = [p for p, _ in items]
    coeffs = [c for _, c in items]
    res = C.cr_frobenius_batch(C.family(3, 5, launch=C.LAUNCH_GRAPH), primes, coeffs, noalloc=True,
                               raise_on_error=False)
    assert res["status"] == C.CR_EINVAL
    mlp = C.Mlp(seed=1)
    try:
        res = C.cr_frobenius_batch(C.family(3, 5, policy=C.CR_POLICY_LEARNED, mlp=mlp), primes, coeffs,
                                   noalloc=True, raise_on_error=False)
        assert res["status"] == C.CR_EINVAL
    finally:
        mlp.close()


def test_noalloc_rejects_a_batch_beyond_the_workspace():
    """Quartic K3 surfaces need far more than the workspace: a clear CR_ENOMEM,
    and the next call still works."""
    k3 = _items("quartic_k3_mixed", range(4))
    res = C.cr_frobenius_batch(C.family(4, 4), [p for p, _ in k3], [c for _, c in k3], noalloc=True,
                               raise_on_error=False)
    assert res["status"] == C.CR_ENOMEM
    assert "static workspace" in C.lib().cr_last_error().decode()
    items = _items("quintic_curves_mixed", range(3))
    fam = C.family(3, 5)
    want = C.cr_frobenius_batch(fam, [p for p, _ in items], [c for _, c in items])
    got = C.cr_frobenius_batch(fam, [p for p, _ in items], [c for _, c in items], noalloc=True)
    _same(got, want)
