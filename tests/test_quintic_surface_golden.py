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
must reproduce the stored matrices bit for bit, on the streaming MFMA kernel
and on the 64-bit VALU kernel.
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


def test_reduced_precision_workload_shares_the_items():
    a, b = workload.WORKLOADS["quintic_surfaces_mixed"], workload.WORKLOADS["quintic_surfaces_r8"]
    assert (a.wid, a.nvars, a.degree, a.primes, a.count) == (b.wid, b.nvars, b.degree, b.primes, b.count)
    assert (b.r, b.n_series) == (8, 2) and (a.r, a.n_series) == (0, 0)
    assert [workload.stream(b, j)[0] for j in range(16)] == [workload.stream(a, j)[0] for j in range(16)]


def test_library_precision_for_the_overrides():
    for it in golden():
        fam = C.family(4, 5, r=it["r"], n_series=it["N"])
        assert C.cr_precision(fam, it["p"]) == (it["r"], it["N"], it["M"])


@pytest.mark.gpu
@pytest.mark.parametrize("engine,policy", [(C.ENGINE_AUTO, C.CR_POLICY_DEPTH_FIRST), (C.ENGINE_AUTO, C.CR_POLICY_P_CHUNK),
                                           (C.ENGINE_VALU, C.CR_POLICY_DEPTH_FIRST)])
def test_gpu_matches_golden_at_reduced_precision(engine, policy):
    """The streaming MFMA kernel (engine 5: 28 quad row tiles x 18 K-blocks,
    base-49 / base-121 digits) and the 64-bit VALU kernel reproduce the
    stored matrices bit for bit."""
    items = golden()
    fam = C.family(4, 5, r=8, n_series=2, engine=engine, policy=policy)
    res = C.cr_frobenius_batch(fam, [it["p"] for it in items], [it["coeffs"] for it in items], raise_on_error=False)
    assert res["stats"].engine == (C.ENGINE_WIDE if engine == C.ENGINE_AUTO else C.ENGINE_VALU)
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


@pytest.mark.gpu
def test_gpu_learned_policy_on_quintic_surfaces_keeps_the_bits():
    """A network trained on the GPU only from the plain p-chunk traces of
    plane quartics, plane quintics and quartic K3 surfaces (no quintic
    surface among them) plans the reductions of the stored quintic surfaces
    at reduced precision: the judge keeps or replaces each plan, and the
    matrices equal the oracle's bit for bit.  The column steps of the learned
    and the p-chunk plans are printed side by side."""
    from tests.gpu_common import workload_items
    xs, ts = [], []
    for nv, d, name, js in [(3, 4, "quartic_curve_f7", [1, 2]), (3, 5, "quintic_curves_mixed", range(300, 303)),
                            (4, 4, "quartic_k3_mixed", [70, 71])]:
        for p, c in workload_items(name, js):
            x, t = C.cr_trace_policy(C.family(nv, d), p, c)
            xs.append(x)
            ts.append(t)
    m = C.Mlp(seed=5)
    losses = m.train(np.concatenate(xs), np.concatenate(ts), epochs=6, batch=1024, lr=2e-3, seed=3)
    assert losses[-1] < losses[0]
    items = golden()
    primes, coeffs = [it["p"] for it in items], [it["coeffs"] for it in items]
    res = C.cr_frobenius_batch(C.family(4, 5, r=8, n_series=2, policy=C.CR_POLICY_LEARNED, mlp=m), primes, coeffs,
                               raise_on_error=False)
    st = res["stats"]
    assert st.policy == C.CR_POLICY_LEARNED and 0 <= st.fallbacks <= len(items)
    pc = sum(C.cr_policy_cost(C.family(4, 5, r=8, n_series=2, policy=C.CR_POLICY_P_CHUNK), p, c).column_steps
             for p, c in zip(primes, coeffs))
    print("quintic surfaces, column steps: learned %d, p-chunk %d (fallbacks %d of %d)"
          % (st.column_steps, pc, st.fallbacks, len(items)), flush=True)
    for i, it in enumerate(items):
        assert [[int(x) for x in row] for row in res["scaled"][i]] == [[int(x) for x in row] for row in it["scaled"]]
        prec = it["col_prec"]
        want = [[int(x) % it["p"] ** prec[c] for c, x in enumerate(row)] for row in it["phi_prime"]]
        assert [[int(x) for x in row] for row in res["frob"][i]] == want
    m.close()


@pytest.mark.gpu
def test_gpu_full_reduced_precision_batch():
    """The whole 16-surface workload at reduced precision: the streaming MFMA
    kernel and the 64-bit VALU kernel give the same scaled matrices, and on
    every surface the trace of Frobenius gives #X(F_p) modulo p^2 (brute-force
    point count)."""
    w = workload.WORKLOADS["quintic_surfaces_r8"]
    fam = C.family(4, 5, r=w.r, n_series=w.n_series)
    items = [workload.first_accepted(w, j, lambda p, c: C.cr_check_smooth(fam, p, c)) for j in range(w.count)]
    primes, coeffs = [p for p, _ in items], [c for _, c in items]
    res = C.cr_frobenius_batch(fam, primes, coeffs, raise_on_error=False)
    assert res["stats"].engine == C.ENGINE_WIDE
    ref = C.cr_frobenius_batch(C.family(4, 5, r=w.r, n_series=w.n_series, engine=C.ENGINE_VALU), primes, coeffs,
                               raise_on_error=False)
    assert ref["stats"].engine == C.ENGINE_VALU
    assert np.array_equal(res["scaled"], ref["scaled"]) and np.array_equal(res["frob"], ref["frob"])
    for i, (p, c) in enumerate(items):
        assert int(res["item_status"][i]) in (C.CR_OK, C.CR_EPRECISION)
        pole = [int(x) for x in res["col_pole"][i]]
        tr = sum(int(res["frob"][i][k][k]) * p ** (3 - pole[k]) for k in range(52))
        f = {e: v % p for e, v in from_coeffs(4, 5, c).items() if v % p}
        assert (1 + p + p * p + tr - count_projective(f, 4, p, 1)) % (p * p) == 0
