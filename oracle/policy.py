"""The reduction game of Section 3.4 played by the policies of Section 4
(test infrastructure only).

Plays the game on exponents alone (the values never matter for its cost):
a term is (u, pole, number of vectors, active basis columns).  Start terms
come from Proposition 2.1 through ``frobenius.start_blocks`` and Tweak
(Algorithm 1); directions come from Algorithm 3; a chunk is the largest k
with u - k v >= 0, capped by the pole orders the phase may still use.

Combining like terms (second move of the game): terms with equal u (hence
equal pole) form a group.  Each term is one vector times a row of column
coefficients, so a group of g terms with active columns A becomes |A|
vectors (one per column) -- done only when g > |A|, so that it never adds
work.  Counters: column steps (cost M each), chunks (cost S each), merged
terms (cost D each), vectors reduced, groups combined, phases.

Policies:
  depth_first  -- Section 4.2: every term straight to pole n, no combining;
  p_chunk      -- Section 4.1: the terms of largest pole L go to max(L - p, n),
                  then like terms are combined; repeat;
  var_by_var   -- Section 4.3: every term until u_c = 0 (c = n, n-1, ..., 0),
                  combining after each variable; the rest goes to pole n.
"""
from collections import defaultdict

from .cohomology import basis
from .frobenius import start_blocks
from .poly import from_coeffs
from .precision import precision_parameters


def greedy_direction(u, d, S):
    """Algorithm 3: a unit on each variable of S that u uses, then round robin
    while v_i < u_i, stopping as soon as |v| = d.  None if |v| stays below d."""
    nv = len(u)
    v = [0] * nv
    left = d
    for s in sorted(S):
        if left and u[s]:
            v[s] = 1
            left -= 1
    while left:
        moved = False
        for m in range(nv):
            if left and v[m] < u[m]:
                v[m] += 1
                left -= 1
                moved = True
        if not moved:
            return None
    return v


def tweak(E, k):
    """Algorithm 1: split k units off the front of E; returns (u, gamma)."""
    u = list(E)
    gam = [0] * len(E)
    for i in range(len(E)):
        t = min(u[i], k)
        u[i] -= t
        gam[i] += t
        k -= t
    return tuple(u), tuple(gam)


def start_terms(nv, d, p, coeffs, S=None):
    """(u0, pole, active columns) of every Proposition 2.1 start term."""
    n = nv - 1
    S = list(range(nv)) if S is None else list(S)
    f = {e: c % p for e, c in from_coeffs(nv, d, coeffs).items() if c % p}
    B = basis(f, nv, d, p)
    r, Nm, sm, M = precision_parameters(p, n, {m: len(B[m]) for m in B})
    q = p ** M
    E, P, coef, _ = start_blocks(f, nv, d, p, S, B, Nm, sm, q)
    out = []
    for e, pole, row in zip(E, P, coef):
        u, _g = tweak(e, d * n - n)
        out.append((u, pole, frozenset(c for c, x in enumerate(row) if int(x) % q)))
    return out


def _run(u, pole, stop, d, S, var, counters):
    """Algorithm 3 chunks from (u, pole) until pole == stop or u[var] == 0."""
    while pole > stop:
        if var is not None and u[var] == 0:
            break
        v = greedy_direction(u, d, S)
        assert v is not None, "no direction of norm d"
        k = min([pole - stop] + [u[i] // v[i] for i in range(len(u)) if v[i]])
        assert k >= 1
        u = tuple(u[i] - k * v[i] for i in range(len(u)))
        pole -= k
        counters["chunks"] += 1
    return u, pole


def _combine(terms, counters):
    groups = defaultdict(list)
    for t in terms:
        groups[t[0]].append(t)
    out = []
    for u, mem in groups.items():
        nvec = sum(t[2] for t in mem)
        cols = frozenset().union(*[t[3] for t in mem])
        if nvec > len(cols):
            counters["combined_groups"] += 1
            counters["merged_terms"] += nvec
            for c in sorted(cols):
                out.append((u, mem[0][1], 1, frozenset([c])))
        else:
            out.extend(mem)
    return out


def play(nv, d, p, starts, policy, S=None):
    """Counters of the game for start terms [(u0, pole, cols)] under `policy`."""
    n = nv - 1
    S = list(range(nv)) if S is None else list(S)
    cnt = defaultdict(int)
    terms = [(u, pole, 1, cols) for (u, pole, cols) in starts]

    def phase(active, stop, var):
        nonlocal terms
        moved = []
        did = False
        for (u, pole, nvec, cols) in active:
            u2, pole2 = _run(u, pole, stop, d, S, var, cnt)
            if pole2 != pole:
                did = True
                cnt["column_steps"] += (pole - pole2) * nvec
                cnt["vectors"] += nvec
            moved.append((u2, pole2, nvec, cols))
        if did:
            cnt["phases"] += 1
        return moved

    if policy == "depth_first":
        phase(terms, n, None)
        return dict(cnt)
    if policy == "p_chunk":
        while True:
            L = max((t[1] for t in terms), default=n)
            if L <= n:
                break
            stop = max(L - p, n)
            act = [t for t in terms if t[1] > stop]
            rest = [t for t in terms if t[1] <= stop]
            moved = phase(act, stop, None)
            terms = [t for t in moved + rest if t[1] > n]
            if terms:
                terms = _combine(terms, cnt)
        return dict(cnt)
    if policy == "var_by_var":
        for var in list(range(nv - 1, -1, -1)) + [None]:
            act = [t for t in terms if t[1] > n and (var is None or t[0][var] != 0)]
            if not act:
                continue
            rest = [t for t in terms if not (t[1] > n and (var is None or t[0][var] != 0))]
            moved = phase(act, n, var)
            terms = [t for t in moved + rest if t[1] > n]
            if not terms:
                break
            terms = _combine(terms, cnt)
        return dict(cnt)
    raise ValueError("unknown policy %r" % policy)
