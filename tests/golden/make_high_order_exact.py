"""Writes high_order_exact.txt: exact operator outputs at sampled nodes of
the order-9 and order-10 parity lattices (40 x 40 jittered, seed 6), from a
40-digit solve of each node's system (oracle/exact.py), next to the float64
oracle's outputs for the same nodes. Uses only the oracle and the seeded
input generator.

    python tests/golden/make_high_order_exact.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from fields import smooth_fields  # noqa: E402
from oracle import exact as X  # noqa: E402
from oracle import labfm_oracle as O  # noqa: E402
from paper_2102_02019_amd import inputs  # noqa: E402

CASES = ((10, 3.2), (9, 3.0))
SAMPLE = tuple(range(7, 1600, 40))


def main():
    lines = ["# Exact (40-digit) and float64-oracle outputs of eq. general_do at sampled",
             "# nodes of the 40x40 jittered lattices (seed 6) at m = 10 (h/s = 3.2) and",
             "# m = 9 (h/s = 3.0), for the fields of tests/fields.py:smooth_fields.",
             "# Written by tests/golden/make_high_order_exact.py (oracle/ only).",
             "# columns: m node field op exact oracle_float64"]
    for m, hs in CASES:
        nodes = inputs.jittered_lattice(40, seed=6, m=m, h_over_s=hs)
        rp, col = O.neighbours(nodes.x, nodes.y, nodes.h, nodes.box)
        fields = smooth_fields(nodes.x, nodes.y)
        names = sorted(fields)
        for i in SAMPLE:
            dx, dy = O.stencil_offsets(nodes.x, nodes.y, nodes.box, rp, col, i)
            c = col[rp[i]:rp[i + 1]]
            dphis = [fields[k][c] - fields[k][i] for k in names]
            ex = X.exact_node_outputs(dx, dy, nodes.h[i], m, dphis)
            w = O.node_weights(dx, dy, nodes.h[i], nodes.s[i], m)["w"]
            for f, k in enumerate(names):
                for d in range(6):
                    orc = float(np.sum(dphis[f] * w[d]))
                    lines.append(f"{m} {i} {k} {d} {float(ex[f, d])!r} {orc!r}")
            print(m, i, flush=True)
    with open(os.path.join(HERE, "high_order_exact.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
