"""Writes the stored expected labels under tests/golden/ using only the CPU oracle.

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# An 8x8 example in the spirit of the paper's running example (Sec. II-A,
# Figs. 1-4, whose pixel values are not recoverable from the text): shapes
# that join only through diagonal contacts, so 4- and 8-connectivity differ.
IMAGE = np.array([
    [0, 1, 1, 0, 0, 1, 1, 0],
    [0, 1, 0, 0, 1, 1, 0, 0],
    [1, 1, 0, 1, 0, 0, 0, 1],
    [0, 0, 0, 0, 1, 1, 0, 1],
    [1, 1, 0, 1, 1, 0, 0, 1],
    [0, 1, 0, 0, 0, 0, 1, 0],
    [0, 0, 1, 1, 0, 1, 1, 0],
    [1, 0, 0, 1, 0, 0, 0, 1],
], dtype=np.uint8)


def block(name, a):
    return "[%s]\n" % name + "\n".join(" ".join("%d" % v for v in row) for row in a) + "\n"


def main():
    l4 = oracle.label(IMAGE, 4)
    l8 = oracle.label(IMAGE, 8)
    with open(os.path.join(HERE, "worked_8x8.txt"), "w") as f:
        f.write("# 8x8 worked example; labels = 1 + smallest raster index (y*8 + x) of the\n")
        f.write("# component, 0 = background.  Written by tests/golden/make_golden.py from the\n")
        f.write("# CPU oracle and checked by hand against the definition (Introduction,\n")
        f.write("# Sec. II-A-3 merge direction).\n")
        f.write(block("image", IMAGE))
        f.write(block("labels_conn4", l4))
        f.write(block("labels_conn8", l8))


if __name__ == "__main__":
    main()
