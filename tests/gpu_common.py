"""Helpers shared by the GPU parity tests (device results vs the CPU oracle)."""
import numpy as np

from oracle.cohomology import is_s_smooth
from oracle.frobenius import frobenius
from oracle.poly import from_coeffs
from paper_2602_24155_amd import crfrob as C
from paper_2602_24155_amd import workload


def oracle_smooth(nv, d):
    def accept(p, c):
        f = {e: v % p for e, v in from_coeffs(nv, d, c).items() if v % p}
        return is_s_smooth(f, nv, d, p, list(range(nv)))
    return accept


def workload_items(name, js):
    w = workload.WORKLOADS[name]
    acc = oracle_smooth(w.nvars, w.degree)
    return [workload.first_accepted(name, j, acc) for j in js]


def assert_item_matches_oracle(res, i, nv, d, p, c, oracle=None):
    """Bit-exact comparison of one batch item with the oracle."""
    o = oracle if oracle is not None else frobenius(nv, d, p, c)
    b = len(o.col_pole)
    assert res["item_status"][i] == 0
    # coordinates before unscaling: exact mod p^M (same for every valid path)
    got = [[int(x) for x in row] for row in res["scaled"][i]]
    want = [[int(x) for x in row] for row in o.scaled]
    assert got == want, "scaled Frobenius coordinates differ (item %d, p=%d)" % (i, p)
    assert [int(x) for x in res["col_pole"][i]] == o.col_pole
    assert [int(x) for x in res["col_prec"][i]] == o.col_prec
    for r_ in range(b):
        for c_ in range(b):
            assert int(res["frob"][i][r_][c_]) == o.phi_prime[r_][c_] % p ** o.col_prec[c_]
    assert res["lpoly"][i] == o.lpoly
    return o


def run_batch(nv, d, items, **kw):
    fam = C.family(nv, d, **kw)
    primes = [p for p, _c in items]
    coeffs = [c for _p, c in items]
    return C.cr_frobenius_batch(fam, primes, coeffs)
