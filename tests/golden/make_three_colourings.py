"""Writes square_three_colourings_m20.txt: P(3) of the square 20 x r
rectangles, r = 1..21, as exact numbers of proper 3-colourings (Sec. 1),
counted by the oracle's colour transfer matrix (oracle/colourings.py), which
shares nothing with the partition transfer matrix.

    python tests/golden/make_three_colourings.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import colourings as OC  # noqa: E402


def main():
    m, n = 20, 21
    counts = OC.square_three_colourings(m, n)
    with open(os.path.join(HERE, "square_three_colourings_m20.txt"), "w") as f:
        f.write("# P(3) of the square m x r rectangle = number of proper 3-colourings (definition, Sec. 1),\n")
        f.write("# by oracle/colourings.py (written by make_three_colourings.py).  Columns: lattice m r q P(q)\n")
        for r, c in enumerate(counts, start=1):
            f.write(f"square {m} {r} 3 {c}\n")


if __name__ == "__main__":
    main()
