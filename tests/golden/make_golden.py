"""Writes the stored expected values under tests/golden/ from the oracle only.

  wells16_k64_brute.txt : the 80 lowest eigenvalues of the 16^3 7-point
                          workload (4 seeded wells, seed 101, h = 0.5) by
                          dense numpy.linalg.eigh of the assembled matrix.
  bloch24_k64_brute.txt : the 80 lowest eigenvalues of the Bloch operator
                          family on a reduced 24^3 grid (13-point, smoothed
                          field seed 103 in [-2, 0], kappa = (2 pi 0.25 / L,
                          0, 0), h = 0.5) by dense numpy.linalg.eigvalsh of
                          the assembled complex Hermitian matrix (about 3
                          minutes and 3 GB).

Run: python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import brute  # noqa: E402
from paper_1407_7506_amd import inputs as I  # noqa: E402


def bloch24():
    p = I.bloch96(N=24, k=64, q=8)
    g = p.grid
    lam = brute.lowest_values(p.V, g.N, g.h, g.order, 80, g.kpt)
    np.savetxt(os.path.join(HERE, "bloch24_k64_brute.txt"), lam, fmt="%.17e",
               header="24^3 13-point Bloch kappa=(2pi*0.25/L,0,0), smoothed field seed 103, h=0.5: "
                      "lowest 80 eigenvalues (dense eigvalsh)")


def main():
    bloch24()
    p = I.wells16()
    lam, _, _ = brute.lowest(p.V, p.grid.N, p.grid.h, p.grid.order, 80)
    np.savetxt(os.path.join(HERE, "wells16_k64_brute.txt"), lam, fmt="%.17e",
               header="16^3 7-point, 4 wells seed 101, h=0.5: lowest 80 eigenvalues (dense eigh)")


if __name__ == "__main__":
    main()
