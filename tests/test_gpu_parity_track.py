"""Running pair histogram: N(r) kept current by the Delta N(r) of every
accepted move (nd_box_track_histogram), and its accumulation over samples
(nd_box_accumulate / nd_box_accumulated).

After every sweep the running counts must equal, bit for bit, both a fresh
nd_pair_histogram of the same coordinates and the FP64 oracle's histogram
of them; the accumulated mean, turned into g(r) and S(Q), must equal the
oracle's mean of the per-sweep g(r) and S(Q) (both are linear in the
counts, so the mean commutes with them).
"""
import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nd():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_1904_08756_amd as nd
    nd.lib()
    return nd


def say(*a):
    print(*a, flush=True)


def _run_tracked(nd, orc, box, T, mcp, seed, dr, nbins, sweeps, trials_per_sweep, check_oracle=True):
    import torch
    g = nd.Box.from_synthetic(box)
    g.set_tables(T.U, T.h, T.r_cut)
    g.track_histogram(dr, nbins)
    V, rho = g.density()
    npairs = orc.pair_counts_total(box.species, box.n_species)
    per_sweep_g = []
    first = 0
    for s in range(sweeps):
        res = g.mc_sweep(mcp, seed, first, trials_per_sweep)
        first += trials_per_sweep
        run = g.tracked_histogram().cpu().numpy().astype(np.uint64)
        fresh = nd.pair_histogram(g, dr, nbins).cpu().numpy().astype(np.uint64)
        assert np.array_equal(run, fresh), f"sweep {s}: running counts differ from a fresh histogram"
        if check_oracle:
            moved = syn.Box(box.name, box.L, box.species, box.unit_offsets, g.coords_host(), box.n_species)
            want, _ = orc.pair_histogram(moved, dr, nbins)
            assert np.array_equal(run, want), f"sweep {s}: running counts differ from the oracle"
        g.accumulate()
        per_sweep_g.append(orc.gr_normalize(run.astype(np.float64), dr, V, npairs))
        say(f"{box.name}: sweep {s}, {res['accepted']} of {trials_per_sweep} accepted, running N(r) exact")
    mean, n = g.accumulated()
    assert n == sweeps
    g_acc = nd.gr_normalize_f64(mean, dr, V, npairs).cpu().numpy()
    g_mean = np.mean(per_sweep_g, axis=0)
    assert np.allclose(g_acc, g_mean, rtol=1e-13, atol=1e-13 * np.abs(g_mean).max())
    torch.cuda.synchronize()
    return g, g_acc, g_mean, V, rho


@pytest.mark.parametrize("k_batch,order,scan", [(0, 0, 0), (1, 0, 0), (64, 0, 0), (0, 1, 0), (0, 0, 1)])
def test_running_histogram_c1(nd, orc, k_batch, order, scan):
    box, T, mc = syn.config_c1()
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"], k_batch=k_batch, order=order, scan=scan)
    g, g_acc, g_mean, V, rho = _run_tracked(nd, orc, box, T, p, mc["seed"], mc["dr"], mc["nbins"], 3, box.n_units)
    if k_batch == 0 and order == 0 and scan == 0:
        # S(Q) of the accumulated g equals the mean of the per-sweep S(Q)
        import torch
        w, self_term = nd.eq1_weights(g, syn.water_b(0.0))
        Q = syn.q_grid()
        S_acc = nd.sq_transform(torch.as_tensor(g_acc, device="cuda"), mc["dr"], rho, w, self_term,
                                torch.as_tensor(Q, device="cuda")).cpu().numpy()
        S_o = orc.sq(g_mean, mc["dr"], rho, w, self_term, Q)
        rk = (np.arange(mc["nbins"]) + 0.5) * mc["dr"]
        scale = float(np.sum(np.abs(w) * 4 * np.pi * rho * np.sum(rk ** 2 * np.abs(g_mean - 1) * mc["dr"], axis=1)))
        assert np.max(np.abs(S_acc - S_o)) <= 1e-11 * (scale + self_term)


def test_running_histogram_units_of_one_to_four_atoms(nd, orc):
    box = syn.mixed_unit_box(400, 19.0, 77, max_atoms=4, n_species=3, name="mixed units")
    T = syn.mixed_tables(r_cut=8.0)
    p = nd.MCParams(2.5, 0.4, 0.3, k_batch=50)
    dr = 0.05
    _run_tracked(nd, orc, box, T, p, 91, dr, syn.n_bins_for(9.4, dr), 3, box.n_units)


def test_running_histogram_sio2_single_atoms_random_order(nd, orc):
    box = syn.atomic_box((2000, 4000), 114.7 * (6000 / 99999) ** (1 / 3), 1003, ("Si", "O"), "SiO2 cut")
    T = syn.sio2_tables()
    p = nd.MCParams(syn.SIO2_MC["kT"], syn.SIO2_MC["max_disp"], 0.0, order=1)
    dr = 0.03
    _run_tracked(nd, orc, box, T, p, 1003, dr, syn.n_bins_for(box.L / 2, dr), 2, box.n_units)


@pytest.mark.timeout(600)
def test_running_histogram_c2_one_sweep(nd, orc):
    """The 99,999-atom water box: one sweep (33,333 trials, about 190 batches)
    with the running histogram, against a fresh histogram and the oracle."""
    import oracle
    oracle.set_threads(oracle.max_threads())
    box, T, mc = syn.config_c2()
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])
    _run_tracked(nd, orc, box, T, p, mc["seed"], mc["dr"], mc["nbins"], 1, box.n_units)


def test_running_histogram_state_errors(nd):
    box, T, mc = syn.config_c1()
    g = nd.Box.from_synthetic(box)
    g.set_tables(T.U, T.h, T.r_cut)
    g._track_nbins = mc["nbins"]
    with pytest.raises(nd.NeudaError, match="STATE"):
        g.tracked_histogram()
    g.track_histogram(mc["dr"], mc["nbins"])
    with pytest.raises(nd.NeudaError, match="STATE"):
        g.accumulated()
    with pytest.raises(nd.NeudaError, match="RANGE"):
        g.track_histogram(mc["dr"], 10 ** 5)
    # new coordinates: the running counts are taken afresh
    rng = np.random.default_rng(3)
    x = box.xyz.copy()
    x[:, :9] = (rng.random((3, 9)) * box.L).astype(np.float32)
    x[x >= box.L] = 0.0
    g.track_histogram(mc["dr"], mc["nbins"])
    g.set_coords(x)
    run = g.tracked_histogram().cpu().numpy()
    fresh = nd.pair_histogram(g, mc["dr"], mc["nbins"]).cpu().numpy()
    assert np.array_equal(run, fresh)
    g.track_histogram(mc["dr"], 0)
