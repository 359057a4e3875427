"""Write the stored expected values used by the GPU parity tests.

Every value here is computed by the FP64 oracle (oracle/) from the seeded
synthetic inputs (synthetic/); nothing comes from the library under test.

  c2_hist.txt   exact pair counts of the 99,999-atom water start
                (33,333 rigid waters, L = 99.7 A, seed 1002), dr = 0.03 A,
                1660 bins, rows O-O, O-H, H-H
  c3_hist.txt   the same for the 99,999-atom SiO2 start (L = 114.7 A,
                seed 1003), 1911 bins, rows Si-Si, Si-O, O-O
  c5_target_sq.txt
                the target S_t(Q) of the differentiated form: a
                99,999-atom water box (33,333 rigid waters, L = 99.7 A,
                seed 1006) run for 10 Metropolis sweeps (seed 1006) with a
                0.5 kJ/mol Gaussian bump of width 0.1 A at r = 2.8 A added
                to the O-O potential; then the Gaussian-broadened histogram
                (sigma 0.02 A, 0.03 A bins to 49.8 A), g(r) and S(Q) at the
                1000-point Q grid with H2O scattering lengths
  f3_hist.txt   exact pair counts of the 1,200,000-atom water start
                (400,000 rigid waters, L = 228.3 A, seed 1007), dr = 0.03 A,
                1660 bins (to 49.8 A)
  c5_hist_broad.txt
                the Gaussian-broadened histogram (sigma 0.02 A, 0.03 A bins,
                1660 bins) of the 99,999-atom water start (seed 1002)

Run: python tests/golden/make_golden.py [hist] [c5] [f3]
(the histograms take about a minute on 8 cores, c5 about fifteen minutes,
f3 about half an hour)
"""
import os
import sys
import time

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


def write_rows(name, header, rows):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        for line in header:
            f.write("# " + line + "\n")
        for row in np.atleast_2d(rows):
            f.write(" ".join(repr(float(x)) for x in row) + "\n")
    print("wrote", path)


def read_rows(name):
    path = os.path.join(HERE, name)
    rows = [[float(x) for x in line.split()] for line in open(path) if not line.startswith("#")]
    return np.array(rows, dtype=np.float64)


def write_c5():
    oracle.set_threads(oracle.max_threads())
    box, T, cfg = syn.config_c5()
    dr, nb, sigma = cfg["dr"], cfg["nbins"], cfg["sigma"]
    # broadened histogram of the differentiated form's own start
    t0 = time.time()
    nh = oracle.hist_broad(box, dr, nb, sigma)
    write_rows("c5_hist_broad.txt", [f"{box.name}: N={box.n_atoms} L={box.L} dr={dr} nbins={nb} sigma={sigma}",
                                     "rows O-O, O-H, H-H; written by the oracle's broadened histogram",
                                     f"({time.time() - t0:.0f} s)"], nh)
    # target: the bumped chain, then the broadened S(Q)
    seed = cfg["target_seed"]
    tbox = syn.water_box(33333, 99.7, seed, "C5 target box")
    Tb = syn.water_tables(emp=syn.oo_bump_emp(0.5, 2.8, 0.1))
    mc = syn.WATER_MC
    xyz = tbox.xyz.copy()
    t0 = time.time()
    res = oracle.mc_run(tbox, Tb, xyz, mc["kT"], mc["max_disp"], mc["max_rot"], seed, 0, 10 * tbox.n_units)
    t_mc = time.time() - t0
    moved = syn.Box("C5 target (after 10 sweeps)", tbox.L, tbox.species, tbox.unit_offsets, xyz, 2)
    nh_t = oracle.hist_broad(moved, dr, nb, sigma)
    V = tbox.L ** 3
    npairs = oracle.pair_counts_total(tbox.species, 2)
    w, self_term = oracle.eq1_weights(tbox.species, 2, syn.water_b(0.0))
    Q = syn.q_grid()
    S_t = oracle.sq(oracle.gr_normalize(nh_t, dr, V, npairs), dr, tbox.n_atoms / V, w, self_term, Q)
    write_rows("c5_target_sq.txt",
               [f"water N={tbox.n_atoms} L={tbox.L} seed {seed}: 10 sweeps ({10 * tbox.n_units} trials, "
                f"{res['n_acc']} accepted, {t_mc:.0f} s) with the O-O bump 0.5 exp(-(r-2.8)^2/(2 0.1^2)) kJ/mol",
                f"then S(Q) of the broadened g (sigma {sigma}, dr {dr}, {nb} bins), H2O weights, "
                f"Q = 0.1 + i 29.9/999, i = 0..999"], S_t)


if __name__ == "__main__":
    which = sys.argv[1:] or ["hist", "c5", "f3"]
    if "hist" in which:
        write_hist("c2_hist.txt", syn.config_c2)
        write_hist("c3_hist.txt", syn.config_c3)
    if "c5" in which:
        write_c5()
    if "f3" in which:
        oracle.set_threads(oracle.max_threads())
        write_hist("f3_hist.txt", lambda: syn.config_scale(400000))
