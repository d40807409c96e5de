"""Writes tests/golden/k3_golden.json: oracle results for three random quartic
K3 surfaces of the quartic_k3_mixed workload (one per prime 7, 11, 13).

Calls only oracle/ (and the seeded input streams); takes a few minutes.
    python tests/golden/make_k3_golden.py
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


def accept(p, c):
    f = {e: v % p for e, v in from_coeffs(4, 4, c).items() if v % p}
    return is_s_smooth(f, 4, 4, p, list(range(4)))


def main():
    out, seen = [], set()
    j = 0
    while len(seen) < 3:
        p, _ = workload.stream("quartic_k3_mixed", j)
        if p not in seen:
            p, c = workload.first_accepted("quartic_k3_mixed", j, accept)
            o = frobenius(4, 4, p, c)
            out.append({"workload": "quartic_k3_mixed", "j": j, "p": p, "coeffs": c,
                        "scaled": [[str(int(x)) for x in row] for row in o.scaled],
                        "col_pole": list(o.col_pole), "col_prec": list(o.col_prec),
                        "phi_prime": [[str(int(x)) for x in row] for row in o.phi_prime],
                        "lpoly": [str(a) for a in o.lpoly]})
            seen.add(p)
            print("j=%d p=%d done" % (j, p), flush=True)
        j += 1
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "k3_golden.json")
    with open(path, "w") as fh:
        json.dump({"source": "oracle.frobenius.frobenius (tests/golden/make_k3_golden.py)", "items": out}, fh)
        fh.write("\n")


if __name__ == "__main__":
    main()
