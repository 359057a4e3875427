"""Throughput of the pair-sum hot path on one MI355X.

One step = the whole hot path on the 99,999-atom water box (33,333 rigid
waters, L = 99.7 A, seeded random start): 10 Metropolis sweeps (333,330
trial moves, each a minimum-image pair sum against every atom), then the
exact pair-count histogram over all 4,999,850,001 pairs (1660 bins of
0.03 A), g(r) and S(Q) at 1000 Q points (Eq. 1).

Prints one JSON line.  `value` is MC moves per second over whole steps
(histogram and S(Q) time included).  Extra fields report the pair-distance
rate, the per-kernel roofline of the dominant kernel (timed with HIP events
inside the timed region), the differentiated form (forward+backward) and
the oracle on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak VALU issue rate of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one non-packed FP32 or FP64 lane operation per lane per clock).
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# Minimum VALU lane operations per distance test of the Metropolis scan:
# 3 sub, 9 nearest image, 3 for r^2, 1 compare with the cutoff.
OPS_PER_TEST = 16
# VALU lane-ops of one exact pair term of a Metropolis trial, as the second
# work unit of the cell scan: 3 sub + 3 for r^2 + 1 compare, 6 for the
# square root (FP32 reciprocal root, FP64 Newton step), 5 for the table
# index and fraction, 3 for the interpolation, 4 for the FP64 sums of U and
# |U|.  A survivor of a trial of a unit of n_u atoms takes 2 n_u of them.
OPS_PER_PAIR_TERM = 25
# wave-level VALU instructions one scan launch of the 99,999-atom water box
# issues (rocprofv3 SQ_INSTS_VALU, profiles/mc_step_water99999.md)
SCAN_ISSUED_WAVE_INSTS = 8.96e6
# Algorithmic VALU lane operations per pair of the exact histogram, as the
# work unit of its roofline: 3 sub, 9 nearest image (mul, round, fma per
# axis), 3 for r^2, 6 for the bin (cvt, sqrt, mul, cvt, edge compare,
# fix-up), 2 range check and address.  The kernel's fixed-point candidate
# path issues about 18 per pair plus the rare exact edge test.
OPS_PER_PAIR = 23
# VALU lane-ops the kernel issues per pair, from rocprofv3 SQ_INSTS_VALU x 64
# / pairs on the same workload (profiles/k_pair_hist_water99999.md)
ISSUED_OPS_PER_PAIR = 21.8
# HBM bytes one k_pair_hist launch moves on the 99,999-atom water box, from
# rocprofv3 FETCH_SIZE / WRITE_SIZE per dispatch scaled by a 1 GiB copy
# (read = 2 x FETCH_SIZE KiB, write = 1 x WRITE_SIZE KiB): 2 x 5130.0 + 19418.5
# KiB.  profiles/k_pair_hist_water99999.md holds the counters and commands;
# set to None whenever the kernel changes until they are taken again.
HIST_TRAFFIC_BYTES = (2 * 5130.5 + 19418.5) * 1024
PAPER_GPU_STEPS_PER_S_1E5 = 12412.0  # Table "tab_speed", water, 1e5 atoms, Tesla V100
# Table "tab_speed", GPU row at the scale-up sizes (atoms: steps/s)
PAPER_GPU_SCALE = {1200000: 3917.0, 3000000: 1963.0, 9999999: 757.0, 30000000: 340.3}


def read_target_sq():
    """S_t(Q) of the differentiated form, stored by tests/golden/make_golden.py
    (the oracle's broadened S(Q) of a water run with an O-O bump)."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "c5_target_sq.txt")
    rows = [[float(x) for x in line.split()] for line in open(path) if not line.startswith("#")]
    return np.array(rows[0])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """Host CPU as lscpu reports it, and the cores this process may use."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            info[k.strip()] = v.strip()
    except Exception:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"model": info.get("Model name"), "sockets": info.get("Socket(s)"),
            "cores_per_socket": info.get("Core(s) per socket"), "threads_per_core": info.get("Thread(s) per core"),
            "cpus": info.get("CPU(s)"), "usable_cpus": usable}


def oracle_step_rate(oracle, box, T, mc, threads, n_mc, n_sub):
    """One thread count: the oracle's Metropolis rate on the first n_mc
    trials and its histogram rate on all pairs of the first n_sub atoms (same
    box, bins and L), combined into the time of one whole step."""
    import numpy as np
    oracle.set_threads(threads)
    used = oracle.max_threads()
    xyz = box.xyz.copy()
    t0 = time.perf_counter()
    oracle.mc_run(box, T, xyz, mc["kT"], mc["max_disp"], mc["max_rot"], mc["seed"], 0, n_mc)
    t_mc = time.perf_counter() - t0
    sub = np.ascontiguousarray(box.xyz[:, :n_sub])
    t0 = time.perf_counter()
    oracle.pair_histogram(sub, mc["dr"], mc["nbins"], L=box.L, species=box.species[:n_sub], n_species=2)
    t_h = time.perf_counter() - t0
    moves_per_s = n_mc / t_mc
    pairs_per_s = n_sub * (n_sub - 1) / 2 / t_h
    n_trials = 10 * box.n_units
    n_pairs = box.n_atoms * (box.n_atoms - 1) / 2
    step_s = n_trials / moves_per_s + n_pairs / pairs_per_s
    return {"value": n_trials / step_s, "threads": used, "mc_moves_per_s": moves_per_s,
            "hist_pairs_per_s": pairs_per_s,
            "sample": (f"{n_mc} Metropolis trials on the 99,999-atom water box ({t_mc:.1f} s) and the exact "
                       f"histogram of its first {n_sub} atoms ({n_sub * (n_sub - 1) // 2} pairs, {t_h:.1f} s)")}


def cpu_baseline(box, T, mc):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    step: once on one thread, once on every core this process may use."""
    import oracle
    cpu = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or cpu["usable_cpus"]
    one = oracle_step_rate(oracle, box, T, mc, 1, 2000, 30000)
    log(f"cpu baseline, 1 thread: {one['value']:.4g} moves/s")
    allc = oracle_step_rate(oracle, box, T, mc, threads, 30000, box.n_atoms)
    log(f"cpu baseline, {allc['threads']} threads: {allc['value']:.4g} moves/s")
    return {
        "value": allc["value"], "unit": "MC moves/s", "cores": allc["threads"], "kind": "oracle",
        "sample": allc["sample"] + "; one whole step's time (10 sweeps + histogram) from the two rates",
        "mc_moves_per_s": allc["mc_moves_per_s"], "hist_pairs_per_s": allc["hist_pairs_per_s"],
        "single_thread": one, "host": cpu,
    }


def batched_leg(nd, syn, np, torch):
    """64 water boxes of log-uniform size (500 to 20,000 molecules, 6 H/D
    weightings): 5 sweeps, histogram, g(r) and S(Q) per box, as one graph
    replay against the same boxes run one by one through the plain calls."""
    sboxes, T4, mc4 = syn.config_c4()
    sweeps, dr = mc4["sweeps"], mc4["dr"]
    params = nd.MCParams(mc4["kT"], mc4["max_disp"], mc4["max_rot"])
    seeds = [mc4["seed"] * 1000 + i for i in range(len(sboxes))]
    nbins = [b.meta["nbins"] for b in sboxes]
    Q = torch.as_tensor(syn.q_grid(), device="cuda")

    def make():
        out = []
        for sb in sboxes:
            g = nd.Box.from_synthetic(sb)
            g.set_tables(T4.U, T4.h, T4.r_cut)
            g.total_energy()
            out.append(g)
        return out

    plain, batched = make(), make()
    w = np.array([nd.eq1_weights(g, syn.water_b(sb.meta["d_fraction"]))[0] for g, sb in zip(plain, sboxes)])
    st = np.array([nd.eq1_weights(g, syn.water_b(sb.meta["d_fraction"]))[1] for g, sb in zip(plain, sboxes)])
    counts = [torch.empty((g.P, nb), dtype=torch.int64, device="cuda") for g, nb in zip(plain, nbins)]
    gr = [torch.empty((g.P, nb), dtype=torch.float64, device="cuda") for g, nb in zip(plain, nbins)]
    sq = [torch.empty(Q.shape[0], dtype=torch.float64, device="cuda") for _ in plain]

    def run_plain(rep):
        for i, g in enumerate(plain):
            g.mc_sweep(params, seeds[i], rep * sweeps * g.n_units, sweeps * g.n_units, stats=False)
            nd.pair_histogram(g, dr, nbins[i], out=counts[i])
            V = g.L * g.L * g.L
            gi = nd.gr_normalize(counts[i], dr, V, nd.pair_counts_total(g))
            nd.sq_transform(gi, dr, g.N / V, w[i], st[i], Q)

    batch = nd.Batch(batched)

    def run_batched(rep):
        batch.run(sweeps, [params] * len(batched), seeds, [rep * sweeps * g.n_units for g in batched], dr,
                  nbins, w, st, Q, counts, gr, sq)

    def timed(fn, reps):
        fn(0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for r in range(1, reps + 1):
            fn(r)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    t_b = timed(run_batched, 3)
    t_p = timed(run_plain, 2)
    moves = sweeps * sum(g.n_units for g in plain)
    pairs = sum(g.N * (g.N - 1) // 2 for g in plain)
    batch.close()
    for b in plain + batched:
        b.close()
    return {
        "tuning": nd.tuning_for("batch", sum(sb.n_atoms for sb in sboxes)),
        "workload": f"{len(sboxes)} water boxes, {sum(g.N for g in plain)} atoms, {sweeps} sweeps each "
                    f"({moves} trials) + histogram ({pairs} pairs) + g(r) + S(Q) at {Q.shape[0]} Q",
        "batched_ms_per_replay": t_b * 1e3, "plain_ms": t_p * 1e3, "speedup": t_p / t_b,
        "batched_mc_moves_per_s": moves / t_b, "plain_mc_moves_per_s": moves / t_p,
        "batched_pairs_per_s": pairs / t_b, "plain_pairs_per_s": pairs / t_p,
    }


def scale_leg(nd, syn, torch, sizes, hist_upto=1_500_000):
    """Water boxes at the C2 density at the sizes of the paper's speed table
    (Table tab_speed: 1.2e6 to 3e7 atoms): Metropolis moves per second over
    200,000 trials after 50,000 warm-up trials, and the exact histogram's
    time where its N^2 pairs take under a few seconds."""
    out = []
    for n_mol in sizes:
        box, T, mc = syn.config_scale(n_mol)
        g = nd.Box.from_synthetic(box)
        g.set_tables(T.U, T.h, T.r_cut)
        p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])
        # the first sweep takes the running energy from cell lists in O(N)
        g.mc_sweep(p, mc["seed"], 0, 50_000, stats=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        g.mc_sweep(p, mc["seed"], 50_000, 200_000, stats=False)
        torch.cuda.synchronize()
        t_mc = time.perf_counter() - t
        rec = {"n_atoms": box.n_atoms, "L": box.L, "mc_moves_per_s": 200_000 / t_mc,
               "paper_gpu_steps_per_s": PAPER_GPU_SCALE.get(box.n_atoms)}
        if box.n_atoms <= hist_upto:
            counts = nd.pair_histogram(g, mc["dr"], mc["nbins"])
            torch.cuda.synchronize()
            t = time.perf_counter()
            nd.pair_histogram(g, mc["dr"], mc["nbins"], out=counts)
            torch.cuda.synchronize()
            t_h = time.perf_counter() - t
            npairs = box.n_atoms * (box.n_atoms - 1) // 2
            # most pairs of a large box lie past the histogram's range and stop
            # at the range test, so no per-pair op count is claimed here
            rec.update(hist_ms=t_h * 1e3, hist_pairs_per_s=npairs / t_h,
                       hist_range_A=mc["dr"] * mc["nbins"])
        g.close()
        del box
        out.append(rec)
        log(f"scale: {rec['n_atoms']} atoms, {rec['mc_moves_per_s']:.3g} moves/s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the forward+backward and SiO2 legs")
    ap.add_argument("--scale-up", action="store_true",
                    help="also the 3e6, 1e7 and 3e7-atom boxes of the paper's speed table (about a minute)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the timed steps, copy a buffer of this many MiB 3 times (a plain copy "
                         "kernel of known size, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the pair-sum path runs on a single MI355X; "
              "a run over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1904_08756_amd as nd
    import synthetic as syn

    torch.cuda.set_device(0)
    box, T, mc = syn.config_c2()
    log(f"bench: {box.name} N={box.n_atoms} L={box.L}")
    g = nd.Box.from_synthetic(box)
    g.set_tables(T.U, T.h, T.r_cut)
    g.total_energy()
    params = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])
    n_trials = mc["n_trials"]
    dr, nbins = mc["dr"], mc["nbins"]
    npairs = nd.pair_counts_total(g)
    V = box.L ** 3
    rho = box.n_atoms / V
    w, self_term = nd.eq1_weights(g, syn.water_b(0.0))
    Q = torch.as_tensor(syn.q_grid(), device="cuda")
    counts = torch.empty((g.P, nbins), dtype=torch.int64, device="cuda")
    # the O(N) scan's distance tests per trial (the paper's per-step work);
    # the cell scan evaluates only the candidates of the cells within reach
    n_tests_per_trial = 2 * 3 * (box.n_atoms - 3)
    n_pairs = box.n_atoms * (box.n_atoms - 1) // 2

    def step(s):
        g.mc_sweep(params, mc["seed"], s * n_trials, n_trials, stats=False)
        nd.pair_histogram(g, dr, nbins, out=counts)
        gr = nd.gr_normalize(counts, dr, V, npairs)
        return nd.sq_transform(gr, dr, rho, w, self_term, Q)

    for s in range(args.warmup):
        step(s)
        torch.cuda.synchronize()
        log(f"warmup step {s} done")
    # timed steps: an event pair around each k_pair_hist launch only (the
    # roofline's kernel time); events around the ~400 Metropolis launches of
    # a step would add a few microseconds to each
    g.set_profiling(True, kernels=("pair_hist",))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.warmup, args.warmup + args.steps):
        S = step(s)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {elapsed:.3f} s")
    hist_n, hist_ms = g.profile("pair_hist")
    g.set_profiling(False)
    assert np.all(np.isfinite(S.cpu().numpy()))
    # kernel time shares: the same number of further steps with an event pair
    # around every launch (not part of the timed figure)
    g.set_profiling(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in range(args.warmup + args.steps, args.warmup + 2 * args.steps):
        step(s)
    torch.cuda.synchronize()
    elapsed_prof = time.perf_counter() - t1
    prof = {k: g.profile(k) for k in ("mc_scan", "mc_corr", "mc_decide", "mc_propose", "pair_hist")}
    g.set_profiling(False)
    log(f"profiled {args.steps} steps in {elapsed_prof:.3f} s")

    # scan work of one more step's sweeps (not timed: counting adds atomics)
    g.count_scan(True)
    g.mc_sweep(params, mc["seed"], (args.warmup + 2 * args.steps) * n_trials, n_trials, stats=False)
    cand, surv = g.count_scan(False)
    torch.cuda.synchronize()
    scan_n, scan_ms = prof["mc_scan"]
    scan_avg_s = scan_ms / max(scan_n, 1) / 1e3
    scan_launch_per_step = scan_n / args.steps
    scan_ops_per_launch = cand * OPS_PER_TEST / scan_launch_per_step
    ms_per_step = 1000.0 * elapsed / args.steps
    moves_per_s = n_trials * args.steps / elapsed
    dist_per_s = (n_trials * n_tests_per_trial + n_pairs) * args.steps / elapsed

    hist_avg_s = hist_ms / max(hist_n, 1) / 1e3
    hist_achieved = n_pairs * OPS_PER_PAIR / hist_avg_s

    result = {
        "metric": "MC moves/s + pair distances/s at 100k atoms; fwd+bwd & batched vs plain",
        "value": moves_per_s,
        "unit": "MC moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": moves_per_s / PAPER_GPU_STEPS_PER_S_1E5,
        "dtype": "f32 pair terms, f64 sums and distances",
        "data": "synthetic (seeded random rigid-water start; no experimental data)",
        "config": {"workload": "water 99,999 atoms (33,333 rigid H2O, L=99.7 A): 10 MC sweeps "
                               "+ exact pair histogram (1660 x 0.03 A bins) + g(r) + S(Q) at 1000 Q",
                   "n_atoms": box.n_atoms, "trials_per_step": n_trials, "pairs_per_step": n_pairs,
                   "parallelism": "single GPU"},
        # dense equivalent: per trial the 2 n_u (N - n_u) tests of the O(N)
        # scan, which the cell scan does not perform; plus every histogram pair
        "dense_equivalent_pair_distances_per_s": dist_per_s,
        "histogram_pair_distances_per_s": n_pairs * args.steps / elapsed,
        # The roofline is taken on the exact pair histogram: its algorithmic
        # work has a fixed definition (every pair once).  The Metropolis
        # kernels evaluate only the pairs their cell neighbourhoods hold, so
        # the per-trial O(N) test count is no measure of their work; their
        # time shares are listed under "kernels".
        "roofline": {
            "kernel": "k_pair_hist (exact pair-count histogram, all N(N-1)/2 pairs)",
            "bound": "alu", "achieved": hist_achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
            "unit": "Tlane-op/s", "frac": hist_achieved / PEAK_LANE_OPS,
            "traffic": HIST_TRAFFIC_BYTES, "traffic_unit": "bytes per launch",
            "launches": hist_n, "avg_launch_ms": hist_avg_s * 1e3,
            "algorithmic_per_launch": f"{n_pairs} pairs x {OPS_PER_PAIR} lane-ops",
            "pairs_per_s": n_pairs / hist_avg_s,
            # the kernel reaches the exact bin with fewer instructions than
            # the algorithmic count (rocprofv3 SQ counters: 21.3 lane-ops
            # issued per pair), so frac can pass 1 while the VALU issue rate
            # stays below its peak
            "issued_lane_ops_per_pair": ISSUED_OPS_PER_PAIR,
            "issued_frac": n_pairs / hist_avg_s * ISSUED_OPS_PER_PAIR / PEAK_LANE_OPS,
        },
        # The Metropolis scan launch (cell scan of a batch's trials, plus the
        # batch's corrections, proposals and final sums): algorithmic work =
        # candidate atoms tested against the trials' reach spheres x 16
        # lane-ops (3 sub, 9 nearest image, 3 for r^2, 1 compare), counted
        # in a further step; time = the launch's average from the profiled steps
        "roofline_mc_scan": {
            "kernel": "k_mc_scan_corr (cell scan of one batch of trials)",
            "bound": "alu", "achieved": scan_ops_per_launch / scan_avg_s / 1e12, "peak": PEAK_LANE_OPS / 1e12,
            "unit": "Tlane-op/s", "frac": scan_ops_per_launch / scan_avg_s / PEAK_LANE_OPS,
            "launches_per_step": scan_launch_per_step, "avg_launch_us": scan_avg_s * 1e6,
            "candidates_per_trial": cand / n_trials, "survivors_per_trial": surv / n_trials,
            "algorithmic_per_launch": f"{cand / scan_launch_per_step:.4g} candidate tests x {OPS_PER_TEST} lane-ops",
            # with the survivors' exact pair terms (2 per atom of the moved
            # unit, old and new) counted too, and the lane-ops the launch
            # issues by the counters
            "frac_with_pair_terms": (scan_ops_per_launch + surv / scan_launch_per_step * 2 * (box.n_atoms / g.n_units)
                                     * OPS_PER_PAIR_TERM)
            / scan_avg_s / PEAK_LANE_OPS,
            "issued_frac": SCAN_ISSUED_WAVE_INSTS * 64 / scan_avg_s / PEAK_LANE_OPS,
        },
        "tuning": nd.tuning_for("box", box.n_atoms),
        "kernels": {
            k: {"launches": n, "ms_total": ms, "share_of_step_time": ms / (1000.0 * elapsed_prof)}
            for k, (n, ms) in prof.items()
        },
        "kernels_note": (f"{args.steps} further steps with an event pair around every launch "
                         f"({1000.0 * elapsed_prof / args.steps:.2f} ms per step with the events)"),
        "paper_context": {"gpu_steps_per_s_1e5_atoms": PAPER_GPU_STEPS_PER_S_1E5,
                          "hardware": "NVIDIA Tesla V100 (Table tab_speed)",
                          "cpu_serial_steps_per_s_1e5_atoms": 62.67},
    }

    if not args.no_extras:
        # differentiated form on the same box: forward (broadened histogram,
        # g, S, chi^2) + backward (adjoint, pair gradient), against the plain
        # histogram + g + S on the same box
        sig = 0.02
        # target S(Q): the oracle's run with the O-O bump (tests/golden/make_golden.py)
        target = torch.as_tensor(read_target_sq(), device="cuda")
        x = torch.as_tensor(g.coords_host(), device="cuda")

        def plain():
            nd.pair_histogram(g, dr, nbins, out=counts)
            return nd.sq_transform(nd.gr_normalize(counts, dr, V, npairs), dr, rho, w, self_term, Q)

        def fwd_bwd():
            xx = x.clone().requires_grad_(True)
            c2 = nd.Chi2Fn.apply(xx, g, dr, nbins, sig, Q, target, syn.water_b(0.0))
            c2.backward()
            return xx.grad

        def timeit(fn, reps=3):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            return float(np.median(ts))

        t_plain = timeit(plain)
        t_fb = timeit(fwd_bwd)
        t_forces = timeit(lambda: nd.forces(g))
        g.set_profiling(True)
        fwd_bwd()
        torch.cuda.synchronize()
        k_fwd = g.profile("hist_broad")[1]
        k_bwd = g.profile("hist_broad_bwd")[1]
        g.set_profiling(False)
        result["forms"] = {
            "plain_hist_g_sq_ms": t_plain * 1e3,
            "fwd_bwd_ms": t_fb * 1e3,
            "fwd_bwd_over_plain": t_fb / t_plain,
            "forces_ms": t_forces * 1e3,
            "fwd_bwd_pairs_per_s": 2 * n_pairs / t_fb,
            "k_hist_broad_ms": k_fwd,
            "k_hist_broad_bwd_ms": k_bwd,
        }
        log("forms done")
        result["forms"]["batched"] = batched_leg(nd, syn, np, torch)
        log("batched done")
        # the paper's O(N) scan (every atom tested for every trial), one sweep
        p_full = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"], scan=nd.ND_SCAN_FULL)
        g.mc_sweep(p_full, mc["seed"], 10 ** 9, 4000, stats=False)
        torch.cuda.synchronize()
        g.set_profiling(True)
        t = time.perf_counter()
        g.mc_sweep(p_full, mc["seed"], 10 ** 9 + 4000, box.n_units, stats=False)
        torch.cuda.synchronize()
        t_full = time.perf_counter() - t
        fn, fms = g.profile("mc_scan")
        g.set_profiling(False)
        f_tests = box.n_units * n_tests_per_trial / fn
        f_avg = fms / fn / 1e3
        result["full_scan"] = {
            "mc_moves_per_s": box.n_units / t_full,
            "roofline": {"kernel": "k_mc_scan (O(N) scan)", "bound": "alu",
                         "achieved": f_tests * OPS_PER_TEST / f_avg / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                         "unit": "Tlane-op/s", "frac": f_tests * OPS_PER_TEST / f_avg / PEAK_LANE_OPS,
                         "frac_packed_peak": f_tests * OPS_PER_TEST / f_avg / (2 * PEAK_LANE_OPS),
                         "launches": fn, "avg_launch_us": f_avg * 1e6,
                         "algorithmic_per_launch": f"{f_tests:.4g} distance tests x {OPS_PER_TEST} lane-ops"},
        }
        log("full scan done")
        # SiO2 box: one sweep of single-atom moves
        box3, T3, mc3 = syn.config_c3()
        g3 = nd.Box.from_synthetic(box3)
        g3.set_tables(T3.U, T3.h, T3.r_cut)
        p3 = nd.MCParams(mc3["kT"], mc3["max_disp"], 0.0)
        g3.mc_sweep(p3, mc3["seed"], 0, 20000, stats=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        g3.mc_sweep(p3, mc3["seed"], 20000, box3.n_units, stats=False)
        torch.cuda.synchronize()
        result["sio2_mc_moves_per_s"] = box3.n_units / (time.perf_counter() - t)
        g3.close()
        log("sio2 done")
        sizes = [400_000] + ([1_000_000, 3_333_333, 10_000_000] if args.scale_up else [])
        result["scale"] = scale_leg(nd, syn, torch, sizes)
        log("scale done")

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["calib_copy_bytes"] = {"read": 4 * n, "write": 4 * n}
        log("copy calibration done")

    # every handle released explicitly while the runtime is up
    g.close()
    torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline(box, T, mc)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
