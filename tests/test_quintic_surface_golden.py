"""Random quintic surfaces (four variables, degree 5: s = 455, J_S from 880
sources to 560 targets) at reduced precision.

Full precision needs p^M up to 2^135, beyond the single-word residues of the
device path (CR_EPRECISION).  At relative precision r = 8 with N_m = 2
series terms (Section 2.5; p^M = 11^9 and 7^9) the whole reduction runs at
the shape of the quintic surfaces, and the oracle finishes in seconds:
tests/golden/quintic_surface_golden.json is written by
tests/golden/make_quintic_surface_golden.py, which calls only oracle/.
On the CPU the stored matrices are pinned by brute-force point counts: the
trace of Frobenius on the primitive H^2, 1 + p + p^2 + tr(Phi) = #X(F_p)
(Section 1.1), holds modulo p^2 at this precision.  On the GPU the library
must reproduce the stored matrices bit for bit.
"""
import json
import os

import numpy as np
import pytest

from oracle.pointcount import count_projective
from oracle.poly import from_coeffs
from paper_2602_24155_amd import crfrob as C
from paper_2602_24155_amd import workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "quintic_surface_golden.json")


def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)["items"]


def test_golden_inputs_are_the_workload_items():
    items = golden()
    assert sorted(it["p"] for it in items) == [7, 11]
    for it in items:
        p, gen = workload.stream("quintic_surfaces_mixed", it["j"])
        assert p == it["p"]
        assert any(next(gen) == it["coeffs"] for _ in range(64))
        assert (it["r"], it["N"], it["M"]) == (8, 2, 9)


def test_golden_trace_matches_point_count_mod_p2():
    for it in golden():
        p = it["p"]
        phi = [[int(x) for x in row] for row in it["phi_prime"]]
        pole = it["col_pole"]
        assert len(phi) == 52 and sorted(set(pole)) == [1, 2, 3]
        assert [pole.count(m) for m in (1, 2, 3)] == [4, 44, 4]
        # Phi = Phi' diag(p^(n - m_c)), n = 3
        tr = sum(phi[c][c] * p ** (3 - pole[c]) for c in range(52))
        f = {e: v % p for e, v in from_coeffs(4, 5, it["coeffs"]).items() if v % p}
        assert (1 + p + p * p + tr - count_projective(f, 4, p, 1)) % (p * p) == 0


def test_library_precision_for_the_overrides():
    for it in golden():
        fam = C.family(4, 5, r=it["r"], n_series=it["N"])
        assert C.cr_precision(fam, it["p"]) == (it["r"], it["N"], it["M"])


@pytest.mark.gpu
def test_gpu_matches_golden_at_reduced_precision():
    items = golden()
    fam = C.family(4, 5, r=8, n_series=2)
    res = C.cr_frobenius_batch(fam, [it["p"] for it in items], [it["coeffs"] for it in items], raise_on_error=False)
    assert res["stats"].engine == C.ENGINE_VALU
    for i, it in enumerate(items):
        assert [[int(x) for x in row] for row in res["scaled"][i]] == [[int(x) for x in row] for row in it["scaled"]]
        assert [int(x) for x in res["col_pole"][i]] == it["col_pole"]
        assert [int(x) for x in res["col_prec"][i]] == it["col_prec"]
        prec = it["col_prec"]
        want = [[int(x) % it["p"] ** prec[c] for c, x in enumerate(row)] for row in it["phi_prime"]]
        assert [[int(x) for x in row] for row in res["frob"][i]] == want


@pytest.mark.gpu
def test_gpu_refuses_full_precision():
    it = golden()[0]
    res = C.cr_frobenius_batch(C.family(4, 5), [it["p"]], [it["coeffs"]], raise_on_error=False)
    assert res["item_status"][0] == C.CR_EPRECISION
