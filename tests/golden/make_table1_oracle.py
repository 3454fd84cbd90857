"""Writes table1_krook_wu_oracle.txt: the oracle's L-infinity errors of
d f^p/dt against the Krook-Wu exact solution for every cell of Table 1
(Sec. 3.2), under the truncation-radius reading R = L/2 = 6 for every pair.

Only the oracle is called.  python tests/golden/make_table1_oracle.py [-j 4]
(about 20 minutes on 4 workers; the N = 56, N_rho = 56 cells dominate).
"""
import argparse
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.krook_wu import table1_errors  # noqa: E402

L, T, R = 12.0, 5.5, 6.0


def printed_cells():
    out = []
    with open(os.path.join(HERE, "table1_krook_wu_all.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            N, Nr, M, ratio = line.split()[:4]
            out.append((int(N), int(Nr), int(M), float(ratio)))
    return out


def one(cell):
    N, Nr, M, ratio = cell
    return cell, table1_errors(N, Nr, M, ratio, L=L, t=T, R=R)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=4)
    args = ap.parse_args()
    cells = printed_cells()
    order = sorted(cells, key=lambda c: -c[0] ** 4 * c[1] * c[2])
    with ProcessPoolExecutor(args.j) as ex:
        res = dict(ex.map(one, order))
    with open(os.path.join(HERE, "table1_krook_wu_oracle.txt"), "w") as fh:
        fh.write("# Oracle errors for Table 1 (written by make_table1_oracle.py from oracle/ only):\n"
                 "# L-infinity error of sum_q Q^{pq} against the Krook-Wu d f^p/dt at t = 5.5\n"
                 "# on [-12, 12]^3, truncation radius R = 6 (= L/2) for every pair.\n"
                 "# Columns: N  N_rho  M  ratio  E1  E2\n")
        for c in cells:
            e1, e2 = res[c]
            fh.write("%d %d %d %g %.6e %.6e\n" % (c + (e1, e2)))


if __name__ == "__main__":
    main()
