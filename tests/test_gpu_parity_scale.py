"""Scale-up to the sizes of the paper's speed table: a 1,200,000-atom water
box (400,000 rigid waters, L = 228.3 A, seed 1007).

* The exact pair histogram of the start (7.2e11 pairs) against the oracle's
  counts, stored by tests/golden/make_golden.py.
* A Metropolis chain of 3,000 trials against the oracle's sequential chain
  trial by trial (each oracle trial is an O(N) pair sum over 1.2e6 atoms).
* The running histogram (Delta N per accepted move) after those trials
  against a fresh histogram of the moved box, bit for bit.
"""
import os
import sys

import numpy as np
import pytest

import synthetic as syn
from helpers import expected_near_ties, f32_ulps

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from make_golden import read_hist  # noqa: E402

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "f3_hist.txt")


@pytest.fixture(scope="module")
def nd():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_1904_08756_amd as nd
    nd.lib()
    return nd


@pytest.fixture(scope="module")
def big(nd):
    box, T, mc = syn.config_scale(400000)
    g = nd.Box.from_synthetic(box)
    g.set_tables(T.U, T.h, T.r_cut)
    return box, T, mc, g


def say(*a):
    print(*a, flush=True)


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="f3_hist.txt not written yet (make_golden.py f3)")
def test_scale_histogram_bit_exact(nd, big):
    box, T, mc, g = big
    say(f"histogram of {box.n_atoms} atoms ({box.n_atoms * (box.n_atoms - 1) // 2} pairs)")
    got = nd.pair_histogram(g, mc["dr"], mc["nbins"]).cpu().numpy().astype(np.uint64)
    want, n_out = read_hist("f3_hist.txt")
    assert np.array_equal(got, want)
    # with the out-of-range pairs the oracle counted, every pair is there once
    npairs = syn.species_counts(box)
    total = np.array([npairs[0] * (npairs[0] - 1) // 2, npairs[0] * npairs[1], npairs[1] * (npairs[1] - 1) // 2],
                     dtype=np.uint64)
    assert np.array_equal(got.sum(axis=1) + n_out, total)


@pytest.mark.timeout(900)
def test_scale_mc_chain_and_running_histogram(nd, orc, big):
    import oracle
    oracle.set_threads(oracle.max_threads())
    box, T, mc, g = big
    g.track_histogram(mc["dr"], mc["nbins"])
    E0 = g.total_energy()
    n = 3000
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])
    say(f"Metropolis chain of {n} trials on {box.n_atoms} atoms")
    res = g.mc_sweep(p, mc["seed"], 0, n, trace=True)
    tr = {k: v.cpu().numpy() for k, v in res["trace"].items()}
    xyz = box.xyz.copy()
    o = orc.mc_run(box, T, xyz, mc["kT"], mc["max_disp"], mc["max_rot"], mc["seed"], 0, n, forced=tr["accepted"])
    assert np.array_equal(tr["unit"], o["unit"])
    assert np.all(np.abs(tr["dE"] - o["dE"]) <= 1e-6 * o["sabs"])
    assert not ((tr["accepted"] != o["acc"]) & (o["tie"] == 0)).any()
    lam = expected_near_ties(o["dE"], o["sabs"], mc["kT"])
    ulps = f32_ulps(g.coords_host(), xyz, box.L)
    say(f"  {int(o['acc'].sum())} accepted, near ties {int(o['tie'].sum())} ({lam:.2f} expected), "
        f"max {int(ulps.max())} ulp")
    assert int(o["tie"].sum()) <= lam + 5.0 * np.sqrt(lam) + 2.0
    assert ulps.max() <= 2
    assert abs((res["E_total"] - E0) - np.sum(o["dE"][o["acc"] == 1])) <= 1e-6 * np.sum(o["sabs"])
    run = g.tracked_histogram().cpu().numpy()
    fresh = nd.pair_histogram(g, mc["dr"], mc["nbins"]).cpu().numpy()
    assert np.array_equal(run, fresh)
    g.track_histogram(mc["dr"], 0)


def test_histogram_counts_past_two_to_the_32(nd):
    """140,000 atoms on two points 5.015 A apart, 70,000 on each: bin 0 holds
    the 2 C(70000, 2) pairs on a point and bin 167 the 70000^2 pairs across,
    both above 2^32, so every carry of a counter into its high word is taken;
    the counts are that closed form, exactly."""
    n = 70000
    xyz = np.full((3, 2 * n), 10.0, np.float32)
    xyz[0, n:] = 15.015
    box = syn.Box("two points", 40.0, np.zeros(2 * n, np.uint8), np.arange(2 * n + 1, dtype=np.int32), xyz, 1)
    g = nd.Box.from_synthetic(box)
    dr, nbins = 0.03, 200
    r = float(np.float32(15.015)) - 10.0
    k = int(r // dr)
    assert (k * dr) ** 2 <= r * r < ((k + 1) * dr) ** 2 and k == 167
    got = nd.pair_histogram(g, dr, nbins).cpu().numpy().astype(np.uint64).ravel()
    want = np.zeros(nbins, np.uint64)
    want[0] = n * (n - 1)
    want[k] = n * n
    assert want[0] > 2 ** 32 and want[k] > 2 ** 32
    assert np.array_equal(got, want)
    g.close()
