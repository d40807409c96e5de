"""Writes tests/golden/quintic_surface_golden.json: the oracle's scaled
Frobenius matrices of two random quintic surfaces of the
quintic_surfaces_mixed workload (one over F_11, one over F_7) at reduced
precision (relative precision r = 8, N_m = 2 series terms; Section 2.5):
the reduction itself at the shape of quintic surfaces (s = 455, J_S from
880 sources to 560 targets), small enough for the oracle.

Calls only oracle/ (and the seeded input streams); about 20 seconds.
    python tests/golden/make_quintic_surface_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.cohomology import is_s_smooth  # noqa: E402
from oracle.frobenius import frobenius  # noqa: E402
from oracle.poly import from_coeffs  # noqa: E402
from paper_2602_24155_amd import workload  # noqa: E402

R, N = 8, 2


def accept(p, c):
    f = {e: v % p for e, v in from_coeffs(4, 5, c).items() if v % p}
    return is_s_smooth(f, 4, 5, p, [0, 1, 2, 3])


def main():
    items = []
    for j in (0, 5):
        p, c = workload.first_accepted("quintic_surfaces_mixed", j, accept)
        o = frobenius(4, 5, p, c, r=R, N=N, lpoly=False)
        items.append({"j": j, "p": p, "coeffs": c, "r": R, "N": N, "M": int(o.M),
                      "scaled": [[str(int(x)) for x in row] for row in o.scaled],
                      "col_pole": list(o.col_pole), "col_prec": list(o.col_prec),
                      "phi_prime": [[str(int(x)) for x in row] for row in o.phi_prime]})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "quintic_surface_golden.json")
    with open(path, "w") as fh:
        json.dump({"source": "oracle.frobenius.frobenius (tests/golden/make_quintic_surface_golden.py)",
                   "items": items}, fh)
        fh.write("\n")


if __name__ == "__main__":
    main()
