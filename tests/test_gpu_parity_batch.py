"""Batched form: water boxes of uneven size and H/D weighting run as one
graph of shared launches.  The full 64-box, 5-sweep workload is checked
against the FP64 oracle box by box (histograms bit for bit, g(r) and S(Q)
at the plain path's tolerances, the Metropolis chains of the smallest boxes
trial by trial); a subset is also checked against the plain entry points
over several graph replays.

Both sides run the same kernels on the same inputs, so coordinates,
histograms, g(r) and acceptance counts agree bit for bit.  The running
energy agrees to rounding (1e-12 relative): the cell scan splits a trial's
pair terms over 1, 2 or 4 waves according to how many trials its launch
holds (one box alone, or every box of a round), and that changes the order
of the FP64 partial sums of a trial's energy change.  S(Q) is held to the
same bound as the plain path (1e-11 of its magnitude scale), and is in
practice identical.  Every plain call is preceded by a reset of
the box's cell lists (set_coords with the box's own coordinates), because
every batched run starts from freshly built cells.
"""
import numpy as np
import pytest

import synthetic as syn
from helpers import expected_near_ties, f32_ulps

pytestmark = pytest.mark.gpu

# smallest three, two in the middle and the largest two of the 64 sizes
PICK = (0, 1, 2, 31, 32, 62, 63)


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


def _subset():
    boxes, T, mc = syn.config_c4()
    order = np.argsort([b.n_atoms for b in boxes], kind="stable")
    return [boxes[int(order[i])] for i in PICK], T, mc


def _make(nd, sboxes, T):
    out = []
    for sb in sboxes:
        g = nd.Box.from_synthetic(sb)
        g.set_tables(T.U, T.h, T.r_cut)
        g.total_energy()
        out.append(g)
    return out


class Setup:
    def __init__(self, nd, sweeps=2):
        import torch
        self.sboxes, self.T, mc = _subset()
        self.mc = mc
        self.sweeps = sweeps
        self.params = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])
        self.seeds = [mc["seed"] * 1000 + i for i in range(len(self.sboxes))]
        self.dr = mc["dr"]
        self.nbins = [sb.meta["nbins"] for sb in self.sboxes]
        self.Q = torch.as_tensor(syn.q_grid(), device="cuda")

    def weights(self, nd, gboxes):
        w, st = [], []
        for sb, g in zip(self.sboxes, gboxes):
            wi, si = nd.eq1_weights(g, syn.water_b(sb.meta["d_fraction"]))
            w.append(wi)
            st.append(si)
        return np.array(w), np.array(st)


def _plain_step(nd, S, gboxes, firsts, w, st):
    res = []
    for i, g in enumerate(gboxes):
        g.set_coords(g.coords(), keep_energy=True)  # fresh cells, as every batched run
        r = g.mc_sweep(S.params, S.seeds[i], firsts[i], S.sweeps * g.n_units)
        counts = nd.pair_histogram(g, S.dr, S.nbins[i])
        V = g.L * g.L * g.L  # the library's own expression for the volume
        gr = nd.gr_normalize(counts, S.dr, V, nd.pair_counts_total(g))
        sq = nd.sq_transform(gr, S.dr, g.N / V, w[i], st[i], S.Q)
        res.append(dict(xyz=g.coords_host(), counts=counts.cpu().numpy(), g=gr.cpu().numpy(),
                        S=sq.cpu().numpy(), accepted=r["accepted"], E=r["E_total"]))
    return res


def _alloc(nd, S, gboxes):
    import torch
    counts = [torch.empty((g.P, nb), dtype=torch.int64, device="cuda") for g, nb in zip(gboxes, S.nbins)]
    gr = [torch.empty((g.P, nb), dtype=torch.float64, device="cuda") for g, nb in zip(gboxes, S.nbins)]
    sq = [torch.empty(S.Q.shape[0], dtype=torch.float64, device="cuda") for _ in gboxes]
    return counts, gr, sq


def _batched_step(S, batch, gboxes, firsts, w, st, outs):
    counts, gr, sq = outs
    stats = batch.run(S.sweeps, [S.params] * len(gboxes), S.seeds, firsts, S.dr, S.nbins, w, st, S.Q,
                      counts, gr, sq, stats=True)
    res = []
    for i, g in enumerate(gboxes):
        res.append(dict(xyz=g.coords_host(), counts=counts[i].cpu().numpy(), g=gr[i].cpu().numpy(),
                        S=sq[i].cpu().numpy(), accepted=stats[i]["accepted"], E=stats[i]["E_total"],
                        trials=stats[i]["trials"]))
    return res


def _compare(a, b, gboxes, sweeps):
    for i, (x, y) in enumerate(zip(a, b)):
        assert y["trials"] == sweeps * gboxes[i].n_units
        assert np.array_equal(x["xyz"], y["xyz"]), f"box {i}: coordinates differ"
        assert x["accepted"] == y["accepted"], f"box {i}"
        assert abs(x["E"] - y["E"]) <= 1e-12 * max(1.0, abs(x["E"])), f"box {i}: {x['E']} vs {y['E']}"
        assert np.array_equal(x["counts"], y["counts"]), f"box {i}: histogram differs"
        assert np.array_equal(x["g"], y["g"]), f"box {i}: g differs"
        scale = np.abs(x["S"]).max() + 1.0
        assert np.max(np.abs(x["S"] - y["S"])) <= 1e-11 * scale, f"box {i}: S differs"


def test_batch_sizes_and_weightings(nd):
    sb, _, _ = _subset()
    n_atoms = [b.n_atoms for b in sb]
    say("batch box atoms", n_atoms)
    assert n_atoms[0] < 2000 and n_atoms[-1] > 40000
    assert len({b.meta["d_fraction"] for b in sb}) >= 3


def test_batch_equals_plain_and_graph_replays(nd):
    import torch
    S = Setup(nd)
    plain = _make(nd, S.sboxes, S.T)
    batched = _make(nd, S.sboxes, S.T)
    w, st = S.weights(nd, plain)
    batch = nd.Batch(batched)
    outs = _alloc(nd, S, batched)
    for rep in range(3):
        firsts = [rep * S.sweeps * g.n_units for g in plain]
        say(f"batch replay {rep}: plain")
        a = _plain_step(nd, S, plain, firsts, w, st)
        say(f"batch replay {rep}: batched")
        b = _batched_step(S, batch, batched, firsts, w, st, outs)
        torch.cuda.synchronize()
        _compare(a, b, batched, S.sweeps)
        say(f"batch replay {rep}: equal; accepted", [x["accepted"] for x in b])
    captures, launches = batch.info()
    assert (captures, launches) == (1, 3)
    batch.close()


def test_batch_histogram_only_and_recapture(nd):
    import torch
    S = Setup(nd)
    gb = _make(nd, S.sboxes[:4], S.T)
    S.sboxes = S.sboxes[:4]
    S.nbins = S.nbins[:4]
    batch = nd.Batch(gb)
    counts = [torch.empty((g.P, nb), dtype=torch.int64, device="cuda") for g, nb in zip(gb, S.nbins)]
    say("batch histogram only")
    batch.run(0, None, None, None, S.dr, S.nbins, counts=counts)
    torch.cuda.synchronize()
    for g, c, nb in zip(gb, counts, S.nbins):
        want = nd.pair_histogram(g, S.dr, nb)
        assert torch.equal(c, want)
    # a different bin count changes the launch structure: captured again
    nb2 = [n - 7 for n in S.nbins]
    counts2 = [torch.empty((g.P, nb), dtype=torch.int64, device="cuda") for g, nb in zip(gb, nb2)]
    batch.run(0, None, None, None, S.dr, nb2, counts=counts2)
    torch.cuda.synchronize()
    for g, c, nb in zip(gb, counts2, nb2):
        assert torch.equal(c, nd.pair_histogram(g, S.dr, nb))
    assert batch.info() == (2, 2)
    batch.close()


def test_batch_rejects_bad_plans(nd):
    import torch
    S = Setup(nd)
    gb = _make(nd, S.sboxes[:2], S.T)
    batch = nd.Batch(gb)
    full = nd.MCParams(S.mc["kT"], S.mc["max_disp"], S.mc["max_rot"], scan=nd.ND_SCAN_FULL)
    with pytest.raises(nd.NeudaError, match="UNSUPPORTED"):
        batch.run(1, [full, full], [1, 2], [0, 0])
    counts = [torch.empty((g.P, 10), dtype=torch.int64, device="cuda") for g in gb]
    with pytest.raises(nd.NeudaError, match="RANGE"):
        batch.run(0, None, None, None, 0.03, [10, 10 ** 6], counts=counts)
    with pytest.raises(nd.NeudaError):
        nd.Batch([gb[0], gb[0]])
    batch.close()



@pytest.mark.timeout(900)
def test_batch_c4_all_boxes_match_oracle(nd):
    """All 64 boxes of the batched workload, 5 sweeps each, then histogram,
    g(r) and S(Q), in one graph replay, against the FP64 oracle: every
    box's counts bit for bit (on the coordinates the batch produced), g to
    1e-14 relative, S(Q) to 1e-11 of the Eq. 1 term scale; the Metropolis
    chains of the three smallest boxes trial by trial against the oracle's
    sequential chain (the chains are cheap there; the others share every
    kernel and launch with them)."""
    import torch

    import oracle
    oracle.set_threads(oracle.max_threads())
    sboxes, T, mc = syn.config_c4()
    sweeps, dr = mc["sweeps"], mc["dr"]
    params = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])
    seeds = [mc["seed"] * 1000 + i for i in range(len(sboxes))]
    nbins = [sb.meta["nbins"] for sb in sboxes]
    Q = torch.as_tensor(syn.q_grid(), device="cuda")
    gb = _make(nd, sboxes, T)
    E0 = [g.energy() for g in gb]
    w, st = [], []
    for sb, g in zip(sboxes, gb):
        wi, si = nd.eq1_weights(g, syn.water_b(sb.meta["d_fraction"]))
        w.append(wi)
        st.append(si)
    w, st = np.array(w), np.array(st)
    batch = nd.Batch(gb)
    counts = [torch.empty((g.P, nb), dtype=torch.int64, device="cuda") for g, nb in zip(gb, nbins)]
    gr = [torch.empty((g.P, nb), dtype=torch.float64, device="cuda") for g, nb in zip(gb, nbins)]
    sq = [torch.empty(Q.shape[0], dtype=torch.float64, device="cuda") for _ in gb]
    say(f"batched C4: {len(gb)} boxes, {sum(g.N for g in gb)} atoms, {sweeps} sweeps")
    stats = batch.run(sweeps, [params] * len(gb), seeds, [0] * len(gb), dr, nbins, w, st, Q, counts, gr, sq,
                      trace=True)
    torch.cuda.synchronize()
    Qh = syn.q_grid()

    # Metropolis chains of the three smallest boxes
    order = np.argsort([g.N for g in gb], kind="stable")
    for i in order[:3]:
        i = int(i)
        sb, g = sboxes[i], gb[i]
        n = sweeps * g.n_units
        tr = {k: v.cpu().numpy() for k, v in stats[i]["trace"].items()}
        xyz = sb.xyz.copy()
        o = oracle.mc_run(sb, T, xyz, mc["kT"], mc["max_disp"], mc["max_rot"], seeds[i], 0, n,
                          forced=tr["accepted"])
        assert np.array_equal(tr["unit"], o["unit"]), f"box {i}: units"
        err = np.abs(tr["dE"] - o["dE"])
        assert np.all(err <= 1e-6 * o["sabs"]), f"box {i}: dE {np.max(err / o['sabs']):.3e}"
        mism = (tr["accepted"] != o["acc"]) & (o["tie"] == 0)
        assert not mism.any(), f"box {i}: decisions differ at {np.nonzero(mism)[0][:10]}"
        # near ties: decisions whose threshold -kT ln u lies within the
        # energy tolerance (1e-6 of the trial's sum of |pair terms|) of dE.
        # Their expected number follows from the exponential law of the
        # threshold; small dense boxes, whose S_abs is large, have several
        n_tie = int(o["tie"].sum())
        lam = expected_near_ties(o["dE"], o["sabs"], mc["kT"])
        assert n_tie <= lam + 5.0 * np.sqrt(lam) + 2.0, f"box {i}: {n_tie} near ties, {lam:.1f} expected"
        ulps = f32_ulps(g.coords_host(), xyz, g.L)
        say(f"box {i} ({g.N} atoms, {n} trials, {int(o['acc'].sum())} accepted): near ties {n_tie} "
            f"({lam:.1f} expected), "
            f"coordinates differing {int((ulps > 0).sum())}, max {int(ulps.max())} ulp")
        assert ulps.max() <= 2, f"box {i}: coordinates {int(ulps.max())} ulp apart"
        dE_acc = np.sum(o["dE"][o["acc"] == 1])
        assert abs((stats[i]["E_total"] - E0[i]) - dE_acc) <= 1e-6 * np.sum(o["sabs"]), f"box {i}: energy"

    # every box: histogram, g(r), S(Q)
    for i, (sb, g) in enumerate(zip(sboxes, gb)):
        moved = syn.Box(sb.name, sb.L, sb.species, sb.unit_offsets, g.coords_host(), 2)
        want, _ = oracle.pair_histogram(moved, dr, nbins[i])
        got = counts[i].cpu().numpy().astype(np.uint64)
        assert np.array_equal(got, want), f"box {i}: histogram differs"
        V = sb.L ** 3
        npairs = oracle.pair_counts_total(sb.species, 2)
        g_o = oracle.gr_normalize(want.astype(np.float64), dr, V, npairs)
        g_d = gr[i].cpu().numpy()
        assert np.all(np.abs(g_d - g_o) <= 1e-14 * np.abs(g_o)), f"box {i}: g"
        w_o, st_o = oracle.eq1_weights(sb.species, 2, syn.water_b(sb.meta["d_fraction"]))
        rho = sb.n_atoms / V
        S_o = oracle.sq(g_o, dr, rho, w_o, st_o, Qh)
        rk = (np.arange(nbins[i]) + 0.5) * dr
        scale = float(np.sum(np.abs(w_o) * 4 * np.pi * rho * np.sum(rk ** 2 * np.abs(g_o - 1.0) * dr, axis=1))) + st_o
        assert np.max(np.abs(sq[i].cpu().numpy() - S_o)) <= 1e-11 * scale, f"box {i}: S(Q)"
    say(f"batched C4: all {len(gb)} boxes equal the oracle")
    batch.close()


def test_batch_random_order_matches_oracle(nd):
    """Random move order in the batched form (units drawn per trial, batches
    cut at the first repeated unit, boxes of different batch counts in one
    graph): the chains of the four smallest boxes trial by trial against
    the oracle."""
    import torch

    import oracle
    sboxes, T, mc = syn.config_c4()
    order = np.argsort([b.n_atoms for b in sboxes], kind="stable")[:4]
    sboxes = [sboxes[int(i)] for i in order]
    gb = _make(nd, sboxes, T)
    E0 = [g.energy() for g in gb]
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"], order=nd.ND_ORDER_RANDOM)
    seeds = [77 + i for i in range(len(gb))]
    batch = nd.Batch(gb)
    sweeps = 2
    stats = batch.run(sweeps, [p] * len(gb), seeds, [5] * len(gb), trace=True)
    torch.cuda.synchronize()
    for i, (sb, g) in enumerate(zip(sboxes, gb)):
        n = sweeps * g.n_units
        tr = {k: v.cpu().numpy() for k, v in stats[i]["trace"].items()}
        xyz = sb.xyz.copy()
        o = oracle.mc_run(sb, T, xyz, mc["kT"], mc["max_disp"], mc["max_rot"], seeds[i], 5, n, order=1,
                          forced=tr["accepted"])
        assert np.array_equal(tr["unit"], o["unit"])
        assert len(np.unique(o["unit"])) < g.n_units
        assert np.all(np.abs(tr["dE"] - o["dE"]) <= 1e-6 * o["sabs"])
        assert not ((tr["accepted"] != o["acc"]) & (o["tie"] == 0)).any()
        ulps = f32_ulps(g.coords_host(), xyz, g.L)
        say(f"random order, box of {g.N} atoms: {int(o['acc'].sum())} of {n} accepted, "
            f"near ties {int(o['tie'].sum())}, max {int(ulps.max())} ulp")
        assert ulps.max() <= 2
        assert abs((stats[i]["E_total"] - E0[i]) - np.sum(o["dE"][o["acc"] == 1])) <= 1e-6 * np.sum(o["sabs"])
    batch.close()
