"""Writes the stored expected values under tests/golden/ by calling the oracle only.

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    X, _ = synth.small(200, 3, 1, kind="mixture", scale=3.0)
    o = oracle.Oracle(X, 10, 4, 1.0)
    perm = o.build_tree()
    with open(os.path.join(HERE, "tree_perm_n200_d3.txt"), "w") as f:
        f.write("# tree permutation of synth.small(200, 3, 1, kind='mixture', scale=3.0), m = 10\n")
        f.write("# (median split along the principal axis; written by make_golden.py from the oracle)\n")
        np.savetxt(f, perm, fmt="%d")


if __name__ == "__main__":
    main()
