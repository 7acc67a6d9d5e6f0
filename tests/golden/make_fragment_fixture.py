"""Writes fragment_pocket.txt: a 12^3 window of sample 12 of the seeded batch
synth.make_batch(64, seed=0) (the first 13 samples are drawn to reach it), centred on
a one-cell contact interface whose only primary neighbour is a fragment that carving
cut off its pore.  Counting pores instead of pore fragments, that interface is not a
dead end and the coarse operator R X P of the window is singular.  The file holds the
image (1 = void), the pore labels and the body force; nothing in it comes from the
solver."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth import make_batch  # noqa: E402


def main():
    w = make_batch(13, seed=0)[12]
    K, J, I, h = 61, 43, 36, 6
    sl = (slice(K - h, K + h), slice(J - h, J + h), slice(I - h, I + h))
    m = w["mask"][sl].astype(np.int64)
    lab = w["labels"][sl].astype(np.int64)
    with open(os.path.join(HERE, "fragment_pocket.txt"), "w") as f:
        f.write("# written by make_fragment_fixture.py: 12^3 window of make_batch(64, seed=0)[12]\n")
        f.write("# shape %d %d %d\n" % m.shape)
        f.write("# body %r %r %r\n" % tuple(float(b) for b in w["body"]))
        np.savetxt(f, np.stack([m.ravel(), lab.ravel()], 1), fmt="%d")


if __name__ == "__main__":
    main()
