"""Writes tsc_cell_centre.txt: the closed-form TSC fractions around a particle at
a cell centre (per-axis weights 1/8, 3/4, 1/8; 3-D weights are products).
Exact rational arithmetic only; no implementation is called."""
import os
from fractions import Fraction as F

HEADER = """# TSC mass fractions around a particle sitting exactly at a cell centre.
# Source: the triangular-shaped-cloud assignment (Hockney & Eastwood) that the
# paper uses for the grid densities (Sect. 2.1, paragraph on the domain grid).
# At the cell centre the per-axis weights are 1/8 (cell i-1), 3/4 (cell i),
# 1/8 (cell i+1); the 3-D weight of cell (i+dx, j+dy, k+dz) is their product:
# 27/64 at the centre, 9/128 on the 6 faces, 3/256 on the 12 edges and
# 1/512 on the 8 corners, summing to 1.
# columns: dx dy dz numerator denominator
"""

if __name__ == "__main__":
    w = {-1: F(1, 8), 0: F(3, 4), 1: F(1, 8)}
    lines = []
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                v = w[dx] * w[dy] * w[dz]
                lines.append(f"{dx} {dy} {dz} {v.numerator} {v.denominator}\n")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tsc_cell_centre.txt")
    with open(path, "w") as fh:
        fh.write(HEADER + "".join(lines))
