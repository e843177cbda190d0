"""Writes square_three_colourings_m<M>.txt for M = 18 and 20: P(3) of the
square M x r rectangles, r = 1..M+1, as exact numbers of proper 3-colourings
(Sec. 1), counted by the oracle's colour transfer matrix
(oracle/colourings.py), which shares nothing with the partition transfer
matrix.

    python tests/golden/make_three_colourings.py [M ...]
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import colourings as OC  # noqa: E402


def write(m: int) -> None:
    n = m + 1
    counts = OC.square_three_colourings(m, n)
    with open(os.path.join(HERE, f"square_three_colourings_m{m}.txt"), "w") as f:
        f.write("# P(3) of the square m x r rectangle = number of proper 3-colourings (definition, Sec. 1),\n")
        f.write("# by oracle/colourings.py (written by make_three_colourings.py).  Columns: lattice m r q P(q)\n")
        for r, c in enumerate(counts, start=1):
            f.write(f"square {m} {r} 3 {c}\n")


def main():
    for m in [int(a) for a in sys.argv[1:]] or [18, 20]:
        write(m)


if __name__ == "__main__":
    main()
