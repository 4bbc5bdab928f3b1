"""Writes the stored expected values under tests/golden/ from the oracle only.

soup_closest_hits.txt: the exhaustive-search closest hits (the plain
definition of closest_hit, Fig. 4 / App. G: the smallest t over every
triangle the FP32 Moller-Trumbore test accepts, ties to the lowest id) of
every 16th ray of the 1,024-triangle soup workload (pinhole camera at
(0.5, 0.5, -1), 64 x 64 rays, seed 1000), as exact float bit patterns.

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2511_15028_amd import workloads as W  # noqa: E402

STRIDE = 16


def soup_rows():
    w = W.soup_workload()
    rays = w["rays"][::STRIDE]
    prim, tuv = oracle.brute_closest(w["verts"], w["tris"], rays)
    rows = []
    for k in range(len(rays)):
        bits = tuv[k].view(np.uint32)
        rows.append(f"{k * STRIDE} {int(prim[k])} {bits[0]:08x} {bits[1]:08x} {bits[2]:08x}")
    return rows


def main():
    with open(os.path.join(HERE, "soup_closest_hits.txt"), "w") as fh:
        fh.write("# closest hits of every 16th ray of the soup workload (1,024 triangles, seed 1000,\n")
        fh.write("# 64 x 64 camera rays), exhaustive search by the oracle (plain definition of\n")
        fh.write("# closest_hit, Fig. 4 / App. G); written by tests/golden/make_golden.py\n")
        fh.write("# columns: ray index, prim id (-1 = miss), t, u, v as IEEE-754 binary32 bits\n")
        for r in soup_rows():
            fh.write(r + "\n")


if __name__ == "__main__":
    main()
