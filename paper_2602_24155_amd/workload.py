"""Seeded synthetic workloads (inputs only; no arithmetic of the method).

Every hypersurface of a workload is drawn from its own NumPy PCG64 stream
seeded with SeedSequence([2602241550 + workload_id, j]): first the prime
(uniform over the workload's primes), then candidate coefficient vectors
(uniform in [0, p), lex-descending monomial order, zeros allowed) until the
consumer accepts one.  Whether a candidate is smooth is decided by the
consumer (the library's own validation, or a reference implementation in
the tests): this module only produces numbers.

A workload may override the precision (r, N_m), for families whose full
precision exceeds the residues of the device path.

The workloads stand in for the paper's random dense hypersurfaces
(Tables 1-2 and Section 6); the paper's example files are not used.  The
sparse workload stands in for the six-term surfaces of Table 2 and the
deformations of Method 2 (Section 6.1): the Fermat hypersurface plus
`extra_terms` random monomials with random nonzero coefficients.
"""
from dataclasses import dataclass
from math import comb

import numpy as np

SEED_BASE = 2602241550


@dataclass(frozen=True)
class Workload:
    wid: int
    name: str
    nvars: int
    degree: int
    primes: tuple
    count: int
    s_mask: int = 0  # 0 = all variables (smooth case)
    extra_terms: int = 0  # > 0: Fermat plus this many random monomials (sparse); 0: dense
    r: int = 0  # relative precision override (0: the precision rule of Section 2.5)
    n_series: int = 0  # series terms N_m override (0: the rule)

    @property
    def ncoeff(self):
        return comb(self.degree + self.nvars - 1, self.nvars - 1)


WORKLOADS = {
    "quartic_curve_f7": Workload(1, "quartic_curve_f7", 3, 4, (7,), 1),
    "quintic_curves_mixed": Workload(2, "quintic_curves_mixed", 3, 5,
                                     (11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47), 256),
    "quintic_curves_p31": Workload(6, "quintic_curves_p31", 3, 5, (31,), 256),
    "quartic_k3_mixed": Workload(3, "quartic_k3_mixed", 4, 4, (7, 11, 13), 64),
    "quintic_surfaces_mixed": Workload(4, "quintic_surfaces_mixed", 4, 5, (7, 11), 16),
    # the same 16 quintic surfaces (same streams) at relative precision 8 with
    # two series terms: p^M = 7^9, 11^9 fit one 64-bit word, where the full
    # precision (p^M up to 2^135) does not
    "quintic_surfaces_r8": Workload(4, "quintic_surfaces_r8", 4, 5, (7, 11), 16, r=8, n_series=2),
    "cubic_fourfold_f7": Workload(5, "cubic_fourfold_f7", 6, 3, (7,), 1, s_mask=1 << 5),
    "sparse_k3_mixed": Workload(7, "sparse_k3_mixed", 4, 4, (7, 11, 13), 64, extra_terms=2),
    "cubic_threefold_f7": Workload(8, "cubic_threefold_f7", 5, 3, (7,), 1, s_mask=1 << 4),
    "cubic_threefolds_mixed": Workload(9, "cubic_threefolds_mixed", 5, 3, (7, 11), 16, s_mask=1 << 4),
}


def monomial_exponents(nvars, degree):
    """Degree-d exponent vectors in the library's order (lexicographically descending)."""
    out = []

    def rec(prefix, left, k):
        if k == nvars - 1:
            out.append(tuple(prefix + [left]))
            return
        for e in range(left, -1, -1):
            rec(prefix + [e], left - e, k + 1)

    rec([], degree, 0)
    return out


def stream(workload, j):
    """(p, generator of candidate coefficient lists) for hypersurface j."""
    w = WORKLOADS[workload] if isinstance(workload, str) else workload
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE + w.wid, j])))
    p = int(w.primes[int(rng.integers(0, len(w.primes)))])

    def gen():
        if w.extra_terms:
            mons = monomial_exponents(w.nvars, w.degree)
            pure = [k for k, m in enumerate(mons) if max(m) == w.degree]
            other = [k for k, m in enumerate(mons) if max(m) < w.degree]
            while True:
                c = [0] * w.ncoeff
                for k in pure:
                    c[k] = 1
                for k in rng.choice(other, size=w.extra_terms, replace=False):
                    c[int(k)] = int(rng.integers(1, p))
                yield c
        while True:
            yield [int(x) for x in rng.integers(0, p, size=w.ncoeff)]

    return p, gen()


def first_accepted(workload, j, accept, max_tries=64):
    """First candidate of hypersurface j for which accept(p, coeffs) is true."""
    p, g = stream(workload, j)
    for _ in range(max_tries):
        c = next(g)
        if accept(p, c):
            return p, c
    raise RuntimeError("no accepted candidate in %d tries" % max_tries)
