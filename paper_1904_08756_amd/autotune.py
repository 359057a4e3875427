"""Autotuner of the library's launch parameters on the GPU at hand.

For each size class it times the candidates on a representative rigid-water
box at liquid density (the workload of the method's Metropolis sweeps and
pair histograms) and keeps the fastest:

  box classes   (nd_mc_sweep, nd_pair_histogram; by the box's atom count)
      up to 10,000 atoms       a 3,000-atom box
      up to 300,000 atoms      the 99,999-atom box
      beyond                   a 1,200,000-atom box
  batch class   (nd_batch_run; by the total atom count of the boxes)
      64 water boxes of 500 to 20,000 molecules (log-uniform), 5 sweeps,
      histograms, g(r) and S(Q) per box, as one graph replay

Searched: the cell scan's waves per trial (1, 2, 4) and the batch target
(expected interacting earlier trials per trial, which sets the Metropolis
batch size) together, timed over whole sweeps; then the pair histogram's
256-thread groups per compute unit with the best of those (4 or 8 for a box:
one or two blocks of four groups sharing a histogram; 3..6 for the batch's
several-box kernel, one group per block).  The result is a text
table (the format of nd_load_tuning) that the binding loads at start-up;
each entry's comment lists the times of every candidate.

Run on the GPU:  python -m paper_1904_08756_amd.autotune --out <file>
and install the file as paper_1904_08756_amd/tuning.txt.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

WAVES = (1, 2, 4)
TARGETS = (9.0, 13.5, 18.0, 27.0, 36.0)
BOX_GROUPS_PER_CU = (4, 8)
BATCH_GROUPS_PER_CU = (3, 4, 5, 6)
BIG = 2 ** 62

BOX_CLASSES = (  # (n_max, molecules of the representative box)
    (10_000, 1_000),
    (300_000, 33_333),
    (BIG, 400_000),
)


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def _timed(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best


def tune_box(nd, syn, torch, n_max, n_mol, quick):
    box, T, mc = syn.config_scale(n_mol, seed=2024 + n_mol)
    g = nd.Box.from_synthetic(box)
    g.set_tables(T.U, T.h, T.r_cut)
    g.total_energy()
    n_trials = min(box.n_units * 2, 200_000)
    nbins = syn.n_bins_for(min(mc["dr"] * mc["nbins"], 0.499 * box.L), mc["dr"])
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])
    counter = [0]

    def sweep():
        g.mc_sweep(p, 11, counter[0], n_trials, stats=False)
        counter[0] += n_trials

    times = {}
    for w in WAVES:
        for tgt in (TARGETS if not quick else (18.0,)):
            nd.set_tuning([dict(kind="box", n_max=BIG, scan_waves=w, batch_target=tgt)])
            times[(w, tgt)] = _timed(torch, sweep, 2)
    w_best, t_best = min(times, key=times.get)
    htimes = {}
    for bpc in BOX_GROUPS_PER_CU:
        nd.set_tuning([dict(kind="box", n_max=BIG, scan_waves=w_best, batch_target=t_best, hist_blocks_per_cu=bpc)])
        htimes[bpc] = _timed(torch, lambda: nd.pair_histogram(g, mc["dr"], nbins), 2)
    b_best = min(htimes, key=htimes.get)
    g.close()
    note = (f"{box.n_atoms} atoms: {n_trials} trials " +
            ", ".join(f"w{w}/t{t:g} {1e3 * s:.2f} ms" for (w, t), s in sorted(times.items())) +
            "; histogram " + ", ".join(f"{b}/CU {1e3 * s:.2f} ms" for b, s in sorted(htimes.items())))
    _log("box class <=", n_max, "->", w_best, t_best, b_best)
    return dict(kind="box", n_max=n_max, scan_waves=w_best, batch_target=t_best, hist_blocks_per_cu=b_best), note


def tune_batch(nd, syn, torch, quick):
    import numpy as np
    sboxes, T, mc = syn.config_c4()
    boxes = []
    for sb in sboxes:
        g = nd.Box.from_synthetic(sb)
        g.set_tables(T.U, T.h, T.r_cut)
        g.total_energy()
        boxes.append(g)
    n_total = sum(g.N for g in boxes)
    params = [nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])] * len(boxes)
    seeds = [mc["seed"] * 1000 + i for i in range(len(boxes))]
    nbins = [sb.meta["nbins"] for sb in sboxes]
    Q = torch.as_tensor(syn.q_grid(), device="cuda")
    w = np.array([nd.eq1_weights(g, syn.water_b(sb.meta["d_fraction"]))[0] for g, sb in zip(boxes, sboxes)])
    st = np.array([nd.eq1_weights(g, syn.water_b(sb.meta["d_fraction"]))[1] for g, sb in zip(boxes, sboxes)])
    counts = [torch.empty((g.P, nb), dtype=torch.int64, device="cuda") for g, nb in zip(boxes, nbins)]
    gr = [torch.empty((g.P, nb), dtype=torch.float64, device="cuda") for g, nb in zip(boxes, nbins)]
    sq = [torch.empty(Q.shape[0], dtype=torch.float64, device="cuda") for _ in boxes]
    batch = nd.Batch(boxes)
    rep = [0]

    def run():
        batch.run(mc["sweeps"], params, seeds, [rep[0] * mc["sweeps"] * g.n_units for g in boxes], mc["dr"], nbins,
                  w, st, Q, counts, gr, sq)
        rep[0] += 1

    times = {}
    for wv in WAVES:
        for tgt in (TARGETS if not quick else (18.0,)):
            nd.set_tuning([dict(kind="batch", n_max=BIG, scan_waves=wv, batch_target=tgt)])
            times[(wv, tgt)] = _timed(torch, run, 3)
    w_best, t_best = min(times, key=times.get)
    htimes = {}
    for bpc in BATCH_GROUPS_PER_CU:
        nd.set_tuning([dict(kind="batch", n_max=BIG, scan_waves=w_best, batch_target=t_best, hist_blocks_per_cu=bpc)])
        htimes[bpc] = _timed(torch, run, 3)
    b_best = min(htimes, key=htimes.get)
    batch.close()
    for g in boxes:
        g.close()
    note = (f"{len(boxes)} boxes, {n_total} atoms, {mc['sweeps']} sweeps + histograms + g + S per replay: " +
            ", ".join(f"w{w}/t{t:g} {1e3 * s:.1f} ms" for (w, t), s in sorted(times.items())) +
            "; histogram " + ", ".join(f"{b}/CU {1e3 * s:.1f} ms" for b, s in sorted(htimes.items())))
    _log("batch ->", w_best, t_best, b_best)
    return dict(kind="batch", n_max=BIG, scan_waves=w_best, batch_target=t_best, hist_blocks_per_cu=b_best), note


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True, help="file to write the tuning table to")
    ap.add_argument("--quick", action="store_true", help="batch target fixed at 18 (fewer candidates)")
    args = ap.parse_args()
    os.environ["NEUDA_NO_TUNING"] = "1"  # start from the built-in choices
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch

    import paper_1904_08756_amd as nd
    import synthetic as syn
    torch.cuda.set_device(0)
    entries, notes = [], []
    for n_max, n_mol in BOX_CLASSES:
        e, note = tune_box(nd, syn, torch, n_max, n_mol, args.quick)
        entries.append(e)
        notes.append(note)
    e, note = tune_batch(nd, syn, torch, args.quick)
    entries.append(e)
    notes.append(note)
    nd.set_tuning([])
    name = torch.cuda.get_device_name(0)
    with open(args.out, "w") as f:
        f.write(f"# neuda tuning table, measured on {name} by paper_1904_08756_amd/autotune.py\n")
        f.write("# kind n_max scan_waves batch_target hist_blocks_per_cu\n")
        for e, note in zip(entries, notes):
            f.write(f"# {note}\n")
            f.write(f"{e['kind']} {e['n_max']} {e['scan_waves']} {e['batch_target']:g} {e['hist_blocks_per_cu']}\n")
    _log("wrote", args.out)


if __name__ == "__main__":
    main()
