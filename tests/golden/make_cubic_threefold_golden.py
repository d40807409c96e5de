"""Writes tests/golden/cubic_threefold_golden.json: the oracle's Frobenius
matrix and L-polynomial of the random cubic threefold of the
cubic_threefold_f7 workload (S = {4}, Definition 3.1; Section 6.5).

Calls only oracle/ (and the seeded input streams); about ten minutes.
    python tests/golden/make_cubic_threefold_golden.py
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

S = [4]


def accept(p, c):
    f = {e: v % p for e, v in from_coeffs(5, 3, c).items() if v % p}
    return is_s_smooth(f, 5, 3, p, S)


def main():
    p, c = workload.first_accepted("cubic_threefold_f7", 0, accept)
    o = frobenius(5, 3, p, c, S=S)
    out = {"workload": "cubic_threefold_f7", "j": 0, "p": p, "S": S, "coeffs": c,
           "scaled": [[str(int(x)) for x in row] for row in o.scaled],
           "col_pole": list(o.col_pole), "col_prec": list(o.col_prec),
           "phi_prime": [[str(int(x)) for x in row] for row in o.phi_prime],
           "lpoly": [str(a) for a in o.lpoly]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cubic_threefold_golden.json")
    with open(path, "w") as fh:
        json.dump({"source": "oracle.frobenius.frobenius (tests/golden/make_cubic_threefold_golden.py)",
                   "items": [out]}, fh)
        fh.write("\n")


if __name__ == "__main__":
    main()
