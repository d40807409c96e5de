"""Brute-force point counts over F_{p^k} (test infrastructure only).

#X(F_q) for X = V(f) in P^n is counted by evaluating f at every point of
P^n(F_q) in the charts [0:..:0:1:*:..:*].  F_q = F_p[x]/(g) with g a primitive
polynomial; elements are integers whose base-p digits are the coefficients of
1, x, x^2, ...; products use discrete-log tables.  This is the definition of
the zeta function's point counts (Section 1.1), with nothing from the
p-adic method.
"""
import itertools

import numpy as np


class GF:
    def __init__(self, p, k):
        self.p, self.k, self.q = p, k, p ** k
        q = self.q
        for tail in itertools.product(range(p), repeat=k):
            g = list(tail) + [1]  # monic: g = x^k + tail[k-1] x^(k-1) + ... + tail[0]
            if g[0] == 0:
                continue
            exp = np.zeros(q - 1, dtype=np.int64)
            cur = [1] + [0] * (k - 1)
            seen = set()
            ok = True
            for i in range(q - 1):
                val = sum(c * p ** j for j, c in enumerate(cur))
                if val in seen:
                    ok = False
                    break
                seen.add(val)
                exp[i] = val
                # multiply by x and reduce modulo g
                top = cur[-1]
                cur = [0] + cur[:-1]
                cur = [(cur[j] - top * g[j]) % p for j in range(k)]
            if ok and len(seen) == q - 1:
                self.exp = exp
                self.log = np.full(q, -1, dtype=np.int64)
                self.log[exp] = np.arange(q - 1)
                return
        raise RuntimeError("no primitive polynomial found")

    def add(self, a, b):
        p = self.p
        out = np.zeros_like(a)
        mul = 1
        for _ in range(self.k):
            out += (((a // mul) % p + (b // mul) % p) % p) * mul
            mul *= p
        return out


def count_projective(coeffs_by_exp, nv, p, k):
    """#{x in P^{nv-1}(F_{p^k}) : f(x) = 0} for f = sum c_e x^e, c_e in Z."""
    F = GF(p, k)
    q = F.q
    terms = [(e, int(c) % p) for e, c in coeffs_by_exp.items() if int(c) % p]
    total = 0
    for lead in range(nv):
        free = nv - lead - 1
        if free == 0:
            grids = []
            npts = 1
        else:
            grids = np.meshgrid(*([np.arange(q, dtype=np.int64)] * free), indexing="ij")
            grids = [g.ravel() for g in grids]
            npts = q ** free
        val = np.zeros(npts, dtype=np.int64)
        for e, c in terms:
            if any(e[i] > 0 for i in range(lead)):
                continue  # leading zeros kill the monomial
            logsum = np.full(npts, int(F.log[c]), dtype=np.int64)
            zero = np.zeros(npts, dtype=bool)
            for t in range(free):
                ei = e[lead + 1 + t]
                if ei == 0:
                    continue
                x = grids[t]
                zero |= (x == 0)
                logsum += ei * np.where(x == 0, 0, F.log[np.maximum(x, 0)])
            term = F.exp[logsum % (q - 1)]
            term = np.where(zero, 0, term)
            val = F.add(val, term)
        total += int(np.count_nonzero(val == 0))
    return total
