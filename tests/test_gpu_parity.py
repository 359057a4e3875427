"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

Histograms are compared bit for bit; energies to 1e-6 of the sum of the
magnitudes of the pair terms involved (the sums are differences of nearly
equal numbers, so a tolerance relative to the result itself would be
meaningless); S(Q) to 1e-11 of the magnitude of the Eq. 1 terms; Metropolis
decisions exactly except inside the near-tie band, where the oracle adopts
the library's decision and the tie is counted.
"""
import math
import os
import sys

import numpy as np
import pytest

import synthetic as syn
from helpers import expected_near_ties, f32_ulps

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


@pytest.fixture(scope="module")
def nd():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_1904_08756_amd as nd
    nd.lib()
    return nd


def _gbox(nd, box, tables=None):
    g = nd.Box.from_synthetic(box)
    if tables is not None:
        g.set_tables(tables.U, tables.h, tables.r_cut)
    return g


def say(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ histogram
def test_histogram_c1_bit_exact(nd, orc):
    box, T, mc = syn.config_c1()
    g = _gbox(nd, box)
    got = nd.pair_histogram(g, mc["dr"], mc["nbins"]).cpu().numpy().astype(np.uint64)
    want, _ = orc.pair_histogram(box, mc["dr"], mc["nbins"])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n,m,L,seed", [(785, 3, 17.0, 1), (2, 1, 5.0, 2), (257, 4, 9.0, 3),
                                        (3 * 256 + 1, 2, 40.0, 4), (5000, 2, 35.0, 5)])
def test_histogram_random_boxes_bit_exact(nd, orc, n, m, L, seed):
    rng = np.random.default_rng(seed)
    xyz = (rng.random((3, n)) * L).astype(np.float32)
    xyz[xyz >= L] = 0.0
    sp = rng.integers(0, m, n).astype(np.uint8)
    sbox = syn.Box("r", L, sp, np.arange(n + 1, dtype=np.int32), xyz, m)
    for dr in (0.1, 0.0371, 0.25):
        nb = syn.n_bins_for(L / 2 * (1 - 1e-6), dr)
        got = nd.pair_histogram(_gbox(nd, sbox), dr, nb).cpu().numpy().astype(np.uint64)
        want, _ = orc.pair_histogram(sbox, dr, nb)
        assert np.array_equal(got, want), (n, m, dr)


def test_histogram_dyadic_edges_and_degenerate_pairs(nd, orc):
    L = 4.0
    pts = [(0.0, 0.0, 0.0), (0.75, 0.0, 0.0), (0.0, 0.0, 0.0), (3.5, 0.0, 0.0), (0.25, 0.5, 0.5),
           (float(np.nextafter(np.float32(4.0), np.float32(0))), 0.0, 0.0), (2.0, 2.0, 2.0),
           (1.75, 0.0, 0.0), (0.5, 0.5, 0.0), (2.0, 0.0, 0.0)]
    xyz = np.array(pts, dtype=np.float32).T.copy()
    n = xyz.shape[1]
    for m in (1, 2):
        sp = (np.arange(n) % m).astype(np.uint8)
        sbox = syn.Box("d", L, sp, np.arange(n + 1, dtype=np.int32), xyz, m)
        got = nd.pair_histogram(_gbox(nd, sbox), 0.25, 7).cpu().numpy().astype(np.uint64)
        want, _ = orc.pair_histogram(sbox, 0.25, 7)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("which", ["c2", "c3"])
def test_histogram_full_size_bit_exact(nd, which):
    from make_golden import read_hist
    cfg = syn.config_c2 if which == "c2" else syn.config_c3
    box, T, mc = cfg()
    want, n_out = read_hist(f"{which}_hist.txt")
    g = _gbox(nd, box)
    got = nd.pair_histogram(g, mc["dr"], mc["nbins"]).cpu().numpy().astype(np.uint64)
    assert np.array_equal(got, want)
    # the same call twice gives the same counts
    got2 = nd.pair_histogram(g, mc["dr"], mc["nbins"]).cpu().numpy().astype(np.uint64)
    assert np.array_equal(got, got2)


def test_histogram_rejects_range_beyond_half_box(nd):
    box, T, mc = syn.config_c1()
    g = _gbox(nd, box)
    with pytest.raises(nd.NeudaError) as e:
        nd.pair_histogram(g, 0.03, 347)  # 10.41 > L/2 = 10.4
    assert e.value.code == -2


# ------------------------------------------------------------------ g(r), S(Q)
def test_gr_and_sq_match_oracle(nd, orc):
    import torch
    box, T, mc = syn.config_c1()
    g = _gbox(nd, box)
    dr, nb = mc["dr"], mc["nbins"]
    counts = nd.pair_histogram(g, dr, nb)
    npairs = nd.pair_counts_total(g)
    assert np.array_equal(npairs, orc.pair_counts_total(box.species, 2))
    V = box.L ** 3
    gr = nd.gr_normalize(counts, dr, V, npairs)
    gr_o = orc.gr_normalize(counts.cpu().numpy().astype(np.float64), dr, V, npairs)
    assert np.allclose(gr.cpu().numpy(), gr_o, rtol=1e-14, atol=0)
    for x in (0.0, 0.64, 1.0):
        w, self_term = nd.eq1_weights(g, syn.water_b(x))
        w_o, self_o = orc.eq1_weights(box.species, 2, syn.water_b(x))
        assert np.allclose(w, w_o, rtol=1e-14) and abs(self_term - self_o) < 1e-13
        Q = torch.as_tensor(syn.q_grid(), device="cuda")
        rho = box.n_atoms / V
        S = nd.sq_transform(gr, dr, rho, w, self_term, Q).cpu().numpy()
        S_o = orc.sq(gr_o, dr, rho, w, self_term, Q.cpu().numpy())
        r = (np.arange(nb) + 0.5) * dr
        scale = np.sum(np.abs(w)[:, None] * 4 * np.pi * rho * r ** 2 * np.abs(gr_o - 1) * dr) + self_o
        assert np.max(np.abs(S - S_o)) <= 1e-11 * scale


def test_sq_flat_for_ideal_gas(nd):
    import torch
    g = torch.ones((3, 400), dtype=torch.float64, device="cuda")
    Q = torch.as_tensor(syn.q_grid(), device="cuda")
    S = nd.sq_transform(g, 0.03, 0.1, [3.7, -9.6, 6.2], 20.545017, Q).cpu().numpy()
    assert np.all(S == 20.545017)


# ------------------------------------------------------------------ energy
@pytest.mark.parametrize("cfg", ["c1", "c3cut"])
def test_total_energy_matches_oracle(nd, orc, cfg):
    if cfg == "c1":
        box, T, _ = syn.config_c1()
    else:
        box = syn.atomic_box((2000, 4000), 114.7 * (6000 / 99999) ** (1 / 3), 1003, ("Si", "O"))
        T = syn.sio2_tables()
    g = _gbox(nd, box, T)
    E = g.total_energy()
    E_o, S_o = orc.total_energy(box, T)
    assert abs(E - E_o) <= 1e-6 * S_o
    assert g.energy() == E


# ------------------------------------------------------------------ Metropolis
def _mc_parity(nd, orc, box, T, params, seed, first, n, k_batch=0, scan=0, order=0):
    g = _gbox(nd, box, T)
    E0 = g.total_energy()
    p = nd.MCParams(params["kT"], params["max_disp"], params["max_rot"], k_batch=k_batch, scan=scan, order=order)
    say(f"mc parity: {box.name} trials {first}..{first + n} K={k_batch} scan={scan} order={order}")
    res = g.mc_sweep(p, seed, first, n, trace=True)
    tr = {k: v.cpu().numpy() for k, v in res["trace"].items()}
    xyz = box.xyz.copy()
    o = orc.mc_run(box, T, xyz, params["kT"], params["max_disp"], params["max_rot"], seed, first, n,
                   forced=tr["accepted"], order=order)
    assert np.array_equal(tr["unit"], o["unit"])
    err = np.abs(tr["dE"] - o["dE"])
    assert np.all(err <= 1e-6 * o["sabs"]), (np.max(err / o["sabs"]), int(np.argmax(err / o["sabs"])))
    mism = (tr["accepted"] != o["acc"]) & (o["tie"] == 0)
    assert not mism.any(), np.nonzero(mism)[0][:10]
    assert res["accepted"] == int(tr["accepted"].sum())
    assert res["trials"] == n
    got_xyz = g.coords_host()
    # identical except where the FP64 sin/cos of the two sides differ in the
    # last place and the rounding to float32 shows it (logged); a unit moved
    # again later carries that ulp along
    ulps = f32_ulps(got_xyz, xyz, box.L)
    n_tie = int(o["tie"].sum())
    lam = expected_near_ties(o["dE"], o["sabs"], params["kT"])
    say(f"  near ties {n_tie} ({lam:.2f} expected); coordinates differing {int((ulps > 0).sum())} "
        f"of {ulps.size}, max {int(ulps.max())} ulp")
    assert n_tie <= lam + 5.0 * np.sqrt(lam) + 2.0
    assert ulps.max() <= 2
    # running energy against a fresh recompute on both sides
    E_run = res["E_total"]
    E_new = g.total_energy()
    E_o, S_o = orc.total_energy(syn.Box("a", box.L, box.species, box.unit_offsets, xyz, box.n_species), T)
    assert abs(E_new - E_o) <= 1e-6 * S_o
    assert abs(E_run - E_new) <= 1e-6 * S_o + 1e-6 * np.sum(o["sabs"])
    assert abs((E_run - E0) - np.sum(o["dE"][o["acc"] == 1])) <= 1e-6 * np.sum(o["sabs"])
    return res, o


@pytest.mark.parametrize("k_batch,scan", [(0, 0), (1, 0), (5, 0), (64, 0), (300, 0), (0, 1), (77, 1)])
def test_mc_c1_matches_sequential_chain(nd, orc, k_batch, scan):
    box, T, mc = syn.config_c1()
    res, o = _mc_parity(nd, orc, box, T, mc, mc["seed"], 0, mc["n_trials"], k_batch, scan)
    assert 0.05 < res["accepted"] / res["trials"] < 0.95


@pytest.mark.parametrize("k_batch,scan", [(0, 0), (9, 0), (0, 1)])
def test_mc_c1_random_order_matches_sequential_chain(nd, orc, k_batch, scan):
    """Units drawn at random per trial (draw 7): batches end before the first
    repeated unit, and the chain still equals the oracle's trial by trial."""
    box, T, mc = syn.config_c1()
    res, o = _mc_parity(nd, orc, box, T, mc, mc["seed"], 0, mc["n_trials"], k_batch, scan, order=1)
    # the draws do repeat units within a sweep's worth of trials
    assert len(np.unique(o["unit"])) < box.n_units
    assert 0.05 < res["accepted"] / res["trials"] < 0.95


def test_mc_sio2_random_order_matches_sequential_chain(nd, orc):
    box = syn.atomic_box((2000, 4000), 114.7 * (6000 / 99999) ** (1 / 3), 1003, ("Si", "O"), "SiO2 cut")
    T = syn.sio2_tables(r_cut=min(12.0, box.L / 2))
    _mc_parity(nd, orc, box, T, syn.SIO2_MC, 1003, 5, 3000, order=1)


def test_mc_c1_split_calls_equal_one_call(nd, orc):
    box, T, mc = syn.config_c1()
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])
    g1 = _gbox(nd, box, T)
    g1.mc_sweep(p, 7, 0, 600)
    g2 = _gbox(nd, box, T)
    g2.mc_sweep(p, 7, 0, 250)
    g2.mc_sweep(p, 7, 250, 350)
    assert np.array_equal(g1.coords_host(), g2.coords_host())


def test_mc_zero_potential_accepts_all(nd):
    box, T, mc = syn.config_c1()
    Z = syn.Tables(np.zeros_like(T.U), T.h, T.r_cut)
    g = _gbox(nd, box, Z)
    res = g.mc_sweep(nd.MCParams(mc["kT"], 0.3, mc["max_rot"]), 3, 0, 500, trace=True)
    assert res["accepted"] == 500
    assert np.all(res["trace"]["dE"].cpu().numpy() == 0.0)


@pytest.mark.parametrize("scan", [0, 1])
def test_mc_c2_sample_matches(nd, orc, scan):
    box, T, mc = syn.config_c2()
    _mc_parity(nd, orc, box, T, mc, mc["seed"], 0, 3000, scan=scan)


@pytest.mark.timeout(900)
def test_mc_c2_full_sweep_matches(nd, orc):
    """One whole sweep of the 99,999-atom water box (33,333 trials, 20
    batches of the bench's size, the cell lists rebuilt at its start) in the
    launch configuration the bench times, against the oracle's sequential
    chain trial by trial."""
    orc.set_threads(orc.max_threads())
    box, T, mc = syn.config_c2()
    res, o = _mc_parity(nd, orc, box, T, mc, mc["seed"], 0, box.n_units)
    assert 0.05 < res["accepted"] / res["trials"] < 0.95


def test_mc_and_histogram_degenerate_boxes(nd, orc):
    """The smallest boxes the boundary accepts: one unit of two atoms (no
    intermolecular pair, so every trial has dE = 0 and is accepted) and two
    one-atom units (a single pair); a call with no trials changes nothing;
    histograms of that one pair, with one bin and with several."""
    T = syn.potential_table(2, 5.0, 0.01, [(3.0, 0.5), (2.5, 0.3)], [0.5, -0.5])
    L = 12.0
    xyz = np.array([[5.0, 5.9], [5.0, 5.4], [5.0, 5.0]], np.float32)
    one = syn.Box("one unit", L, np.array([0, 1], np.uint8), np.array([0, 2], np.int32), xyz.copy(), 2)
    two = syn.Box("two units", L, np.array([0, 1], np.uint8), np.array([0, 1, 2], np.int32), xyz.copy(), 2)
    params = dict(kT=2.5, max_disp=0.5, max_rot=0.3)
    res, _ = _mc_parity(nd, orc, one, T, params, 21, 0, 64)
    assert res["accepted"] == 64
    _mc_parity(nd, orc, two, T, params, 22, 0, 200)
    g = _gbox(nd, two, T)
    E0 = g.total_energy()
    before = g.coords_host()
    res0 = g.mc_sweep(nd.MCParams(2.5, 0.5, 0.3), 5, 0, 0)
    assert res0["trials"] == 0 and res0["accepted"] == 0
    assert np.array_equal(g.coords_host(), before) and g.energy() == E0
    for nbins, dr in ((1, 5.9), (20, 0.25)):
        got = nd.pair_histogram(g, dr, nbins).cpu().numpy()
        want, _ = orc.pair_histogram(two, dr, nbins)
        assert np.array_equal(got, want) and got.sum() == 1
    g.close()


def test_mc_c2_later_trials_match(nd, orc):
    box, T, mc = syn.config_c2()
    # start mid-sweep: trial numbers far from 0 use the same counter-based draws
    _mc_parity(nd, orc, box, T, mc, mc["seed"], 1_000_003, 1500)


@pytest.mark.parametrize("scan", [0, 1])
def test_mc_c3_sample_matches(nd, orc, scan):
    box, T, mc = syn.config_c3()
    _mc_parity(nd, orc, box, T, mc, mc["seed"], 0, 4000, scan=scan)


def test_mc_cells_rebuild_across_sweeps(nd, orc):
    """A run longer than one sweep rebuilds the cells between batches; small
    box, many sweeps: the chain still matches the oracle trial by trial."""
    box = syn.water_box(120, 16.0, 31, "rebuild")
    T = syn.water_tables(r_cut=7.0)
    params = dict(kT=syn.kT_at(298.0), max_disp=0.3, max_rot=math.radians(10.0))
    _mc_parity(nd, orc, box, T, params, 5, 0, 120 * 6, k_batch=50)


@pytest.mark.parametrize("k_batch,scan", [(0, 0), (7, 0), (0, 1)])
def test_mc_mixed_unit_sizes_match(nd, orc, k_batch, scan):
    """Units of 1 to 4 atoms and three species (the widest unit template),
    units straddling the box faces, r_cut + 2 rad < L/2."""
    box = syn.mixed_unit_box(600, 30.0, 77)
    T = syn.mixed_tables()
    params = dict(kT=syn.kT_at(298.0), max_disp=0.25, max_rot=math.radians(12.0))
    _mc_parity(nd, orc, box, T, params, 11, 0, 1500, k_batch=k_batch, scan=scan)


def test_mc_mixed_units_small_box(nd, orc):
    """Same mix where r_cut + 2 rad >= L/2 (every pair takes its own image)."""
    box = syn.mixed_unit_box(150, 17.0, 78)
    T = syn.mixed_tables()
    params = dict(kT=syn.kT_at(298.0), max_disp=0.25, max_rot=math.radians(12.0))
    _mc_parity(nd, orc, box, T, params, 12, 0, 600)


def test_mc_scan_modes_agree(nd):
    box, T, mc = syn.config_c2()
    p_c = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"], scan=0)
    p_f = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"], scan=1)
    g1 = _gbox(nd, box, T)
    g2 = _gbox(nd, box, T)
    r1 = g1.mc_sweep(p_c, 9, 0, 40000, trace=True)
    r2 = g2.mc_sweep(p_f, 9, 0, 40000, trace=True)
    d1 = r1["trace"]["dE"].cpu().numpy()
    d2 = r2["trace"]["dE"].cpu().numpy()
    s1 = r1["trace"]["sabs"].cpu().numpy()
    a1 = r1["trace"]["accepted"].cpu().numpy()
    a2 = r2["trace"]["accepted"].cpu().numpy()
    # identical decisions (a differing near tie would show up here first)
    assert np.array_equal(a1, a2)
    assert np.all(np.abs(d1 - d2) <= 1e-6 * s1)


def test_mc_rejects_missing_tables(nd):
    box, T, mc = syn.config_c1()
    g = _gbox(nd, box)
    with pytest.raises(nd.NeudaError) as e:
        g.mc_sweep(nd.MCParams(mc["kT"], 0.3, 0.1), 1, 0, 10)
    assert e.value.code == -5


def test_profiling_mask_selects_kernels(nd):
    # events only around the kernels of the mask; the others launch bare
    box, T, mc = syn.config_c1()
    g = _gbox(nd, box, T)
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])
    g.set_profiling(True, kernels=("pair_hist",))
    g.mc_sweep(p, 3, 0, box.n_units)
    nd.pair_histogram(g, mc["dr"], mc["nbins"])
    n_scan, ms_scan = g.profile("mc_scan")
    n_hist, ms_hist = g.profile("pair_hist")
    g.set_profiling(False)
    assert (n_scan, ms_scan) == (0, 0.0)
    assert n_hist == 1 and ms_hist > 0.0
    g.set_profiling(True)
    g.mc_sweep(p, 3, box.n_units, box.n_units)
    assert g.profile("mc_scan")[0] > 0 and g.profile("mc_decide")[0] > 0
    g.set_profiling(False)
    # a bit past the kernel ids is an error
    assert nd.lib().nd_box_set_profiling_mask(g.handle, 1 << 8) == -1  # ND_E_INVALID


# ------------------------------------------------------------------ differentiated form
def _broad_box():
    return syn.water_box(600, 18.0, 21, "broad")


def test_hist_broad_matches_oracle(nd, orc):
    box = _broad_box()
    dr, sigma = 0.03, 0.02
    nb = syn.n_bins_for(9.0 * (1 - 1e-6), dr)
    got = nd.hist_broad(_gbox(nd, box), dr, nb, sigma).cpu().numpy()
    want = orc.hist_broad(box, dr, nb, sigma)
    assert np.all(np.abs(got - want) <= 1e-6 * np.maximum(want, 1.0)), np.max(np.abs(got - want))
    # total mass: every pair whose window lies inside the binned range adds 1
    assert abs(got.sum() - want.sum()) <= 1e-9 * want.sum()


def test_hist_broad_backward_matches_oracle(nd, orc):
    import torch
    box = _broad_box()
    dr, sigma = 0.03, 0.02
    nb = syn.n_bins_for(9.0 * (1 - 1e-6), dr)
    rng = np.random.default_rng(2)
    A = rng.normal(size=(3, nb))
    got = nd.hist_broad_backward(_gbox(nd, box), dr, nb, sigma, torch.as_tensor(A, device="cuda")).cpu().numpy()
    want = orc.hist_broad_backward(box, dr, nb, sigma, A)
    scale = np.abs(want).max()
    assert np.all(np.abs(got - want) <= 1e-5 * scale + 1e-4 * np.abs(want)), np.max(np.abs(got - want)) / scale


@pytest.mark.parametrize("sigma", [0.006, 0.036])
def test_hist_broad_other_widths(nd, orc, sigma):
    # both take the forward's tail-mass path (sigma = 0.006 A: dr/sigma = 5,
    # too sharp for the bin-mass table; 0.036 A: 6 sigma = 7.2 dr, too wide
    # for it); at 0.006 A the backward evaluates each edge's density directly
    # (no recurrence)
    import torch
    box = _broad_box()
    dr = 0.03
    nb = syn.n_bins_for(8.5 * (1 - 1e-6), dr)
    g = _gbox(nd, box)
    got = nd.hist_broad(g, dr, nb, sigma).cpu().numpy()
    want = orc.hist_broad(box, dr, nb, sigma)
    assert np.all(np.abs(got - want) <= 1e-6 * np.maximum(want, 1.0)), np.max(np.abs(got - want))
    A = np.random.default_rng(3).normal(size=(3, nb))
    gb = nd.hist_broad_backward(g, dr, nb, sigma, torch.as_tensor(A, device="cuda")).cpu().numpy()
    wb = orc.hist_broad_backward(box, dr, nb, sigma, A)
    scale = np.abs(wb).max()
    assert np.all(np.abs(gb - wb) <= 1e-5 * scale + 1e-4 * np.abs(wb)), np.max(np.abs(gb - wb)) / scale


def test_hist_broad_backward_repeatable_and_nonfinite(nd, orc):
    # integer sums: two calls agree bit for bit; a non-finite adjoint gives
    # NaN everywhere instead of a silently wrong gradient
    import torch
    box = _broad_box()
    dr, sigma = 0.03, 0.02
    nb = syn.n_bins_for(8.5 * (1 - 1e-6), dr)
    g = _gbox(nd, box)
    A = torch.as_tensor(np.random.default_rng(5).normal(size=(3, nb)), device="cuda")
    g1 = nd.hist_broad_backward(g, dr, nb, sigma, A).cpu().numpy()
    g2 = nd.hist_broad_backward(g, dr, nb, sigma, A).cpu().numpy()
    assert np.array_equal(g1, g2)
    A[1, nb // 2] = float("inf")
    g3 = nd.hist_broad_backward(g, dr, nb, sigma, A).cpu().numpy()
    assert np.all(np.isnan(g3))
    A[1, nb // 2] = float("nan")
    g4 = nd.hist_broad_backward(g, dr, nb, sigma, A).cpu().numpy()
    assert np.all(np.isnan(g4))
    A[1, nb // 2] = 0.0
    g5 = nd.hist_broad_backward(g, dr, nb, sigma, A).cpu().numpy()
    assert np.all(np.isfinite(g5))


@pytest.mark.parametrize("kind,n,L,seed", [("atoms", 2, 5.0, 31), ("atoms", 5, 7.0, 32), ("mixed", 180, 12.0, 33),
                                           ("atoms", 513, 14.0, 34)])
def test_differentiated_small_and_ragged_boxes(nd, orc, kind, n, L, seed):
    # the broadened histogram, its backward and the forces on boxes of a
    # few atoms (one mostly empty tile), rigid units of 1-4 atoms with 3
    # species, and 513 atoms (one atom past the last full tile of 512 and
    # of 256)
    import torch
    if kind == "atoms":
        box = syn.atomic_box([n - n // 2, n // 2], L, seed)
        T = syn.potential_table(2, round(0.45 * L, 2), 0.01, [(3.0, 0.5), (3.4, 0.3)], [0.5, -0.3])
    else:
        box = syn.mixed_unit_box(n, L, seed)
        T = syn.mixed_tables(r_cut=round(0.45 * L, 2))
    dr, sigma = 0.05, 0.03
    nb = syn.n_bins_for(0.45 * L, dr)
    g = _gbox(nd, box, T)
    got = nd.hist_broad(g, dr, nb, sigma).cpu().numpy()
    want = orc.hist_broad(box, dr, nb, sigma)
    assert np.all(np.abs(got - want) <= 1e-6 * np.maximum(want, 1.0)), np.max(np.abs(got - want))
    A = np.random.default_rng(seed).normal(size=want.shape)
    gb = nd.hist_broad_backward(g, dr, nb, sigma, torch.as_tensor(A, device="cuda")).cpu().numpy()
    wb = orc.hist_broad_backward(box, dr, nb, sigma, A)
    scale = max(np.abs(wb).max(), 1e-300)
    assert np.all(np.abs(gb - wb) <= 1e-5 * scale + 1e-4 * np.abs(wb)), np.max(np.abs(gb - wb)) / scale
    gf, E = nd.forces(g)
    wf, E_o = orc.forces(box, T)
    fscale = max(np.abs(wf).max(), 1e-300)
    assert np.all(np.abs(gf.cpu().numpy() - wf) <= 1e-9 * fscale + 1e-9 * np.abs(wf))
    _, S_t = orc.total_energy(box, T)
    assert abs(E - E_o) <= 1e-9 * max(S_t, 1e-300)


def test_forces_resolve_small_gradients(nd, orc):
    # the steep short-range end of the table (r_min = 0.5 A, a step of
    # ~1e11 kJ/mol/A) sets the integer scale of the gradient sums; a lone
    # pair far from it (r = 3.2 A, gradient ~1 kJ/mol/A) is still resolved
    # to 1e-9 of its size
    L = 12.0
    xyz = np.array([[1.0, 4.2], [2.0, 2.0], [3.0, 3.0]], dtype=np.float32)
    box = syn.Box("pair", L, np.zeros(2, dtype=np.uint8), np.arange(3, dtype=np.int32), xyz, 1)
    T = syn.potential_table(1, 5.0, 0.01, [(3.0, 0.5)], [0.0])
    gf, E = nd.forces(_gbox(nd, box, T))
    wf, E_o = orc.forces(box, T)
    assert np.abs(wf).max() > 0.1
    assert np.all(np.abs(gf.cpu().numpy() - wf) <= 1e-9 * np.abs(wf).max())
    assert abs(E - E_o) <= 1e-12 * abs(E_o)


def test_forces_repeatable(nd, orc):
    # integer gradient sums and a fixed energy order: repeated calls agree bit for bit
    box = syn.water_box(600, 18.0, 22, "forces")
    T = syn.water_tables(r_cut=9.0)
    g = _gbox(nd, box, T)
    g1, E1 = nd.forces(g)
    g2, E2 = nd.forces(g)
    assert np.array_equal(g1.cpu().numpy(), g2.cpu().numpy()) and E1 == E2


def test_forces_match_oracle(nd, orc):
    box = syn.water_box(600, 18.0, 22, "forces")
    T = syn.water_tables(r_cut=9.0)
    grad, E = nd.forces(_gbox(nd, box, T))
    grad = grad.cpu().numpy()
    want, E_o = orc.forces(box, T)
    scale = np.abs(want).max()
    assert np.all(np.abs(grad - want) <= 1e-9 * scale + 1e-9 * np.abs(want))
    E_t, S_t = orc.total_energy(box, T)
    assert abs(E - E_o) <= 1e-9 * S_t


def test_chi2_autograd_matches_oracle(nd, orc):
    import torch
    box = _broad_box()
    dr, sigma = 0.03, 0.02
    nb = syn.n_bins_for(9.0 * (1 - 1e-6), dr)
    Q = syn.q_grid(300)
    b = syn.water_b(0.0)
    target = 20.0 + 0.5 * np.sin(Q)
    g = _gbox(nd, box)
    # FP64 coordinates (float32-representable): the gradient comes back in FP64
    x = torch.as_tensor(box.xyz.astype(np.float64), device="cuda").clone().requires_grad_(True)
    c2 = nd.Chi2Fn.apply(x, g, dr, nb, sigma, torch.as_tensor(Q, device="cuda"),
                         torch.as_tensor(target, device="cuda"), b)
    # the box moves on before backward runs: the gradient is still taken at x
    other = box.xyz.copy()
    other[0] = np.float32(0.5) * other[0]
    g.set_coords(other)
    c2.backward()
    assert x.grad.dtype == torch.float64
    nh = orc.hist_broad(box, dr, nb, sigma)
    npairs = orc.pair_counts_total(box.species, 2)
    V = box.L ** 3
    w, self_term = orc.eq1_weights(box.species, 2, b)
    S = orc.sq(orc.gr_normalize(nh, dr, V, npairs), dr, box.n_atoms / V, w, self_term, Q)
    chi2_o = float(((S - target) ** 2).sum())
    assert abs(float(c2.detach()) - chi2_o) <= 1e-6 * chi2_o
    A = orc.sq_adjoint(2 * (S - target), nb, dr, box.n_atoms / V, V, w, npairs, Q)
    want = orc.hist_broad_backward(box, dr, nb, sigma, A)
    got = x.grad.cpu().numpy()
    scale = np.abs(want).max()
    # the bound of the direct backward test: FP32 pair weights, FP64 sums
    assert np.all(np.abs(got - want) <= 1e-5 * scale + 1e-4 * np.abs(want)), np.max(np.abs(got - want)) / scale


def test_energy_autograd_gives_forces(nd, orc):
    import torch
    box = syn.water_box(300, 16.0, 23, "eg")
    T = syn.water_tables(r_cut=8.0)
    g = _gbox(nd, box, T)
    x = torch.as_tensor(box.xyz, device="cuda").clone().requires_grad_(True)
    E = nd.EnergyFn.apply(x, g)
    E.backward()
    want, E_o = orc.forces(box, T)
    scale = np.abs(want).max()
    assert np.all(np.abs(x.grad.cpu().numpy() - want) <= 1e-6 * scale + 1e-6 * np.abs(want))


# ------------------------------------------------------------------ boundary
def test_sweep_after_new_coordinates_reports_fresh_energy(nd, orc):
    """A sweep after set_coords (or after the differentiated form loaded its
    own coordinates) starts from the energy of the new configuration."""
    box, T, mc = syn.config_c1()
    g = _gbox(nd, box, T)
    g.total_energy()
    rng = np.random.default_rng(5)
    moved = box.xyz.copy()
    moved[:, :30] = (rng.random((3, 30)) * box.L).astype(np.float32)
    moved[moved >= box.L] = 0.0
    g.set_coords(moved)
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])
    res = g.mc_sweep(p, mc["seed"], 0, 300)
    E_fresh = g.total_energy()
    _, S_o = orc.total_energy(box, T)
    assert abs(res["E_total"] - E_fresh) <= 1e-6 * S_o


def test_device_coordinates_are_wrapped_and_checked(nd):
    import torch
    box, T, mc = syn.config_c1()
    g = _gbox(nd, box, T)
    x = torch.as_tensor(box.xyz.astype(np.float64), device="cuda")
    shifted = x.clone()
    shifted[0, :10] += box.L        # one period up
    shifted[1, 10:20] -= 2 * box.L  # two periods down
    g.set_coords(shifted)
    got = g.coords_host()
    want = box.xyz.astype(np.float64)
    d = np.abs(got.astype(np.float64) - want)
    d = np.minimum(d, box.L - d)
    assert np.all(got >= 0) and np.all(got < box.L)
    assert d.max() < 1e-5
    before = g.coords_host()
    bad = x.clone()
    bad[2, 7] = float("nan")
    with pytest.raises(nd.NeudaError, match="INVALID"):
        g.set_coords(bad)
    assert np.array_equal(g.coords_host(), before)


def test_box_density(nd):
    box, _, _ = syn.config_c1()
    g = _gbox(nd, box)
    V, rho = g.density()
    assert V == box.L * box.L * box.L and rho == box.n_atoms / V


@pytest.mark.parametrize("which", ["c1", "c2", "sio2", "mixed"])
def test_energy_refresh_from_cells_equals_all_pairs(nd, orc, which):
    """A sweep of zero trials after new coordinates reports the energy that
    the sweep recomputes from cell lists in O(N); it equals the all-pairs
    total (the same pair terms, summed in another order)."""
    if which == "c1":
        box, T, mc = syn.config_c1()
    elif which == "c2":
        box, T, mc = syn.config_c2()
    elif which == "sio2":
        box = syn.atomic_box((2000, 4000), 114.7 * (6000 / 99999) ** (1 / 3), 1003, ("Si", "O"), "SiO2 cut")
        T = syn.sio2_tables()
    else:
        box = syn.mixed_unit_box(400, 19.0, 77, max_atoms=4, n_species=3, name="mixed units")
        T = syn.mixed_tables(r_cut=8.0)
    g = _gbox(nd, box, T)
    g.set_coords(box.xyz)  # running energy stale
    res = g.mc_sweep(nd.MCParams(2.5, 0.1, 0.0), 1, 0, 0)
    E_all = g.total_energy()
    if box.n_atoms <= 10000:
        _, S = orc.total_energy(box, T)
    else:
        S = abs(E_all) * 10.0
    say(f"{which}: cells {res['E_total']!r} all pairs {E_all!r}")
    assert abs(res["E_total"] - E_all) <= 1e-12 * S
