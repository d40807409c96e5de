"""Seeded input generators and the search driver's candidates (host only)."""
import numpy as np

from paper_2602_24155_amd import crfrob as C
from paper_2602_24155_amd import search, workload


def test_monomial_order_is_the_library_order():
    for nv, d in ((3, 4), (3, 5), (4, 4), (4, 5), (6, 3)):
        assert [tuple(int(x) for x in m) for m in C.cr_monomials(nv, d)] == workload.monomial_exponents(nv, d)


def test_sparse_workload_is_fermat_plus_two_terms():
    w = workload.WORKLOADS["sparse_k3_mixed"]
    mons = workload.monomial_exponents(4, 4)
    for j in range(8):
        p, g = workload.stream(w, j)
        c = next(g)
        assert p in (7, 11, 13)
        assert all(c[k] == 1 for k, m in enumerate(mons) if max(m) == 4)
        extra = [k for k, m in enumerate(mons) if max(m) < 4 and c[k]]
        assert len(extra) == 2 and all(1 <= c[k] < p for k in extra)


def test_search_candidates_are_smooth():
    rng = np.random.Generator(np.random.PCG64(3))
    fam = C.family(4, 4)
    for method in (1, 2):
        cs = search.candidates(4, 4, 7, 4, rng, method=method, extra_terms=1)
        assert len(cs) == 4 and all(C.cr_check_smooth(fam, 7, c) for c in cs)
        if method == 2:
            assert all(sum(1 for x in c if x) == 5 for c in cs)
