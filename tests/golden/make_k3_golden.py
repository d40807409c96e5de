"""Writes tests/golden/k3_golden.json: oracle results for random quartic K3
surfaces of the quartic_k3_mixed workload, the first four of each prime
7, 11, 13 in workload order.

Calls only oracle/ (and the seeded input streams); about a minute and a half
per surface, run on a pool of host processes.
    python tests/golden/make_k3_golden.py
"""
import json
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.cohomology import is_s_smooth  # noqa: E402
from oracle.frobenius import frobenius  # noqa: E402
from oracle.poly import from_coeffs  # noqa: E402
from paper_2602_24155_amd import workload  # noqa: E402

PER_PRIME = 4


def accept(p, c):
    f = {e: v % p for e, v in from_coeffs(4, 4, c).items() if v % p}
    return is_s_smooth(f, 4, 4, p, list(range(4)))


def one(j):
    p, c = workload.first_accepted("quartic_k3_mixed", j, accept)
    o = frobenius(4, 4, p, c)
    print("j=%d p=%d done" % (j, p), flush=True)
    return {"workload": "quartic_k3_mixed", "j": j, "p": p, "coeffs": c,
            "scaled": [[str(int(x)) for x in row] for row in o.scaled],
            "col_pole": list(o.col_pole), "col_prec": list(o.col_prec),
            "phi_prime": [[str(int(x)) for x in row] for row in o.phi_prime],
            "lpoly": [str(a) for a in o.lpoly]}


def main():
    js, count = [], {7: 0, 11: 0, 13: 0}
    j = 0
    while min(count.values()) < PER_PRIME:
        p, _ = workload.stream("quartic_k3_mixed", j)
        if count[p] < PER_PRIME:
            js.append(j)
            count[p] += 1
        j += 1
    with mp.get_context("fork").Pool(min(len(js), os.cpu_count() or 1)) as pool:
        out = pool.map(one, js, chunksize=1)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "k3_golden.json")
    with open(path, "w") as fh:
        json.dump({"source": "oracle.frobenius.frobenius (tests/golden/make_k3_golden.py)", "items": out}, fh)
        fh.write("\n")


if __name__ == "__main__":
    main()
