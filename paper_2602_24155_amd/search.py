"""Random search for hypersurfaces with a prescribed Newton polygon (Section 6.1).

Method 1 draws random dense equations; Method 2 keeps a fixed equation (here
the Fermat hypersurface, supersingular when p^k = -1 mod d) and adds random
monomials with random nonzero coefficients.  Each round computes the zeta
functions of a batch of smooth candidates on the GPU (cr_frobenius_batch,
one batched call) and classifies their Newton polygons (cr_newton_polygon);
the hypersurfaces whose invariants satisfy the caller's predicate are kept.
Everything numeric runs in the library; this module only draws candidates
and filters results.
"""
import numpy as np

from . import crfrob as C
from .workload import monomial_exponents


def candidates(nvars, degree, p, count, rng, method=1, extra_terms=2, s_mask=0):
    """`count` smooth coefficient lists (the library's monomial order) drawn by
    Method 1 (dense, uniform in F_p) or Method 2 (Fermat plus `extra_terms`
    random monomials)."""
    fam = C.family(nvars, degree, s_mask)
    mons = monomial_exponents(nvars, degree)
    pure = [k for k, m in enumerate(mons) if max(m) == degree]
    other = [k for k, m in enumerate(mons) if max(m) < degree]
    out, tries = [], 0
    while len(out) < count:
        tries += 1
        if tries > 1000 * count:
            raise RuntimeError("too few smooth candidates")
        if method == 1:
            c = [int(x) for x in rng.integers(0, p, size=len(mons))]
        else:
            c = [0] * len(mons)
            for k in pure:
                c[k] = 1
            for k in rng.choice(other, size=extra_terms, replace=False):
                c[int(k)] = int(rng.integers(1, p))
        if C.cr_check_smooth(fam, p, c):
            out.append(c)
    return out


def invariants(nvars, degree, p, lpoly):
    """Newton-polygon record of one Q(T) as a dict."""
    r = C.cr_newton_polygon(nvars, degree, p, C.lpoly_words(lpoly))
    return {"slopes": [(int(r.seg_rise[k]), int(r.seg_len[k])) for k in range(r.nseg)], "p_rank": r.p_rank,
            "ordinary": bool(r.ordinary), "supersingular": bool(r.supersingular),
            "height": None if r.height < 0 else (float("inf") if r.height == 0 else r.height),
            "domino": None if r.domino_num < 0 else r.domino_num / r.domino_den}


def search(nvars, degree, p, want, count=64, rounds=1, seed=0, method=1, extra_terms=2,
           policy=C.CR_POLICY_P_CHUNK, stream=None):
    """Candidates in `rounds` batches of `count`; returns (found, seen): found
    lists dicts {coeffs, lpoly, invariants} whose invariants satisfy
    want(invariants), seen the invariants of every candidate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fam = C.family(nvars, degree, policy=policy)
    found, seen = [], []
    for _ in range(rounds):
        cand = candidates(nvars, degree, p, count, rng, method, extra_terms)
        res = C.cr_frobenius_batch(fam, [p] * len(cand), cand, stream=stream, want_scaled=False)
        for c, a in zip(cand, res["lpoly"]):
            inv = invariants(nvars, degree, p, a)
            seen.append(inv)
            if want(inv):
                found.append({"coeffs": c, "lpoly": a, "invariants": inv})
    return found, seen
