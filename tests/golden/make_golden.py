"""Write the stored expected values used by the GPU parity tests.

Every value here is computed by the FP64 oracle (oracle/) from the seeded
synthetic inputs (synthetic/); nothing comes from the library under test.

  c2_hist.txt   exact pair counts of the 99,999-atom water start
                (33,333 rigid waters, L = 99.7 A, seed 1002), dr = 0.03 A,
                1660 bins, rows O-O, O-H, H-H
  c3_hist.txt   the same for the 99,999-atom SiO2 start (L = 114.7 A,
                seed 1003), 1911 bins, rows Si-Si, Si-O, O-O

Run: python tests/golden/make_golden.py   (about a minute on 8 cores)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synthetic as syn  # noqa: E402


def write_hist(name, cfg):
    box, _, mc = cfg()
    counts, n_out = oracle.pair_histogram(box, mc["dr"], mc["nbins"])
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        f.write(f"# {box.name}: N={box.n_atoms} L={box.L} dr={mc['dr']} nbins={mc['nbins']}\n")
        f.write("# pairs beyond the last bin per pair type: " + " ".join(str(int(x)) for x in n_out) + "\n")
        for row in counts:
            f.write(" ".join(str(int(x)) for x in row) + "\n")
    print("wrote", path)


def read_hist(name):
    path = os.path.join(HERE, name)
    rows, n_out = [], None
    for line in open(path):
        if line.startswith("# pairs beyond"):
            n_out = np.array([int(x) for x in line.split(":")[1].split()], dtype=np.uint64)
        elif not line.startswith("#"):
            rows.append([int(x) for x in line.split()])
    return np.array(rows, dtype=np.uint64), n_out


if __name__ == "__main__":
    write_hist("c2_hist.txt", syn.config_c2)
    write_hist("c3_hist.txt", syn.config_c3)
