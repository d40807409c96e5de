"""CPU oracle for controlled reduction (TEST INFRASTRUCTURE ONLY).

This package is a plain, slow, independent implementation of what the
controlled-reduction hot path computes: the Frobenius matrix of a smooth
projective hypersurface over F_p (7 <= p < 50) modulo p^M and its integer
L-polynomial.  It follows the paper's Section 2 (cohomology basis, Frobenius
expansion of Proposition 2.1, precision), Section 3 (Proposition 3.3 and the
explicit formula for R_{u,v}, Algorithm 1 Tweak) and Section 4 (Algorithm 3
greedy choice of v) literally, with polynomial arithmetic on exact integers
and a small plain-C inner loop for speed.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this package.  The
product path (``paper_2602_24155_amd``) never imports it and shares no code,
tables or constants with it.

Parity status of each function is stated in its docstring; every function is
pinned by tests under ``tests/test_oracle_*.py`` against brute-force point
counts, closed forms (Weil's Gauss/Jacobi-sum formula for diagonal
hypersurfaces, supersingular Fermat curves), the functional equation, the
Riemann hypothesis bound and invariance properties.
"""
