"""Flexible molecules on the GPU against the oracle: intramolecular
harmonic terms between every two atoms of a unit (nd_box_set_intra) and
single-atom moves mixed with whole-molecule moves (atom_frac, atom_disp;
Sec. "Correctness").  Per-trial energy changes to 1e-6 of the sum of the
magnitudes of their terms, every decision outside the near-tie band, final
coordinates to the last float32 place; total energy and forces with the
intramolecular part; the running Delta N(r) histogram and the batched form
with single-atom moves."""
import math

import numpy as np
import pytest

import synthetic as syn
from helpers import expected_near_ties, f32_ulps

pytestmark = pytest.mark.gpu

K_WATER = np.array([0.0, 2000.0, 600.0])  # kJ/mol/A^2: O-O (none inside a water), O-H, H-H


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


def _distorted(n_mol, L, seed):
    box = syn.water_box(n_mol, L, seed, "flexible water")
    r0_box = syn.Box(box.name, box.L, box.species, box.unit_offsets, box.xyz.copy(), 2)
    rng = np.random.default_rng(seed)
    x = box.xyz.astype(np.float64) + rng.normal(scale=0.03, size=box.xyz.shape)
    box.xyz = np.ascontiguousarray((x - L * np.floor(x / L)).astype(np.float32))
    box.xyz[box.xyz >= L] = 0.0
    return box, r0_box


def _gbox(nd, box, ref, T):
    """A GPU machine whose reference geometry is `ref`, then moved to box's coordinates."""
    g = nd.Box.from_synthetic(ref)
    g.set_tables(T.U, T.h, T.r_cut)
    g.set_intra(K_WATER)
    g.set_coords(box.xyz)
    return g


@pytest.mark.parametrize("k_batch,scan,order", [(0, 0, 0), (7, 0, 0), (0, 1, 0), (0, 0, 1)])
def test_flexible_chain_matches_oracle(nd, orc, k_batch, scan, order):
    box, ref = _distorted(300, 20.8, 1001)
    T = syn.water_tables()
    r0 = orc.intra_reference(ref)
    g = _gbox(nd, box, ref, T)
    E0 = g.total_energy()
    Ei, Si = orc.intra_energy(box, K_WATER, r0)
    Eo, So = orc.total_energy(box, T)
    assert abs(E0 - (Eo + Ei)) <= 1e-6 * (So + Si)
    mc = syn.WATER_MC
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"], k_batch=k_batch, scan=scan, order=order,
                    atom_frac=0.5, atom_disp=0.05)
    n = 1500
    res = g.mc_sweep(p, 31, 0, n, trace=True)
    tr = {k: v.cpu().numpy() for k, v in res["trace"].items()}
    xyz = box.xyz.copy()
    o = orc.mc_run_flex(box, T, xyz, mc["kT"], mc["max_disp"], mc["max_rot"], 0.5, 0.05, K_WATER, r0, 31, 0, n,
                        order=order, forced=tr["accepted"])
    assert np.array_equal(tr["unit"], o["unit"])
    assert np.all(np.abs(tr["dE"] - o["dE"]) <= 1e-6 * o["sabs"])
    assert not ((tr["accepted"] != o["acc"]) & (o["tie"] == 0)).any()
    lam = expected_near_ties(o["dE"], o["sabs"], mc["kT"])
    assert int(o["tie"].sum()) <= lam + 5 * np.sqrt(lam) + 2
    ulps = f32_ulps(g.coords_host(), xyz, box.L)
    n_atom = int((o["atom"] >= 0).sum())
    say(f"flexible chain K={k_batch} scan={scan} order={order}: {n_atom} atom moves of {n}, "
        f"{int(o['acc'].sum())} accepted, max {int(ulps.max())} ulp")
    assert 0.3 * n < n_atom < 0.7 * n
    assert ulps.max() <= 2
    E1 = g.total_energy()
    Ei1, Si1 = orc.intra_energy(syn.Box("m", box.L, box.species, box.unit_offsets, xyz, 2), K_WATER, r0)
    Eo1, So1 = orc.total_energy(syn.Box("m", box.L, box.species, box.unit_offsets, xyz, 2), T)
    assert abs(E1 - (Eo1 + Ei1)) <= 1e-6 * (So1 + Si1)
    assert abs(res["E_total"] - E1) <= 1e-6 * (So1 + Si1) + 1e-6 * np.sum(o["sabs"])


def test_flexible_forces_match_oracle(nd, orc):
    box, ref = _distorted(200, 16.0, 8)
    T = syn.water_tables(r_cut=8.0)
    r0 = orc.intra_reference(ref)
    g = _gbox(nd, box, ref, T)
    grad, E = nd.forces(g)
    want, E_o = orc.forces(box, T)
    want = want + orc.intra_forces(box, K_WATER, r0)
    Ei, _ = orc.intra_energy(box, K_WATER, r0)
    scale = np.abs(want).max()
    assert np.all(np.abs(grad.cpu().numpy() - want) <= 1e-9 * scale + 1e-9 * np.abs(want))
    _, S_t = orc.total_energy(box, T)
    assert abs(E - (E_o + Ei)) <= 1e-9 * S_t + 1e-9 * abs(Ei)


def test_flexible_running_histogram(nd, orc):
    box, ref = _distorted(300, 20.8, 12)
    T = syn.water_tables()
    g = _gbox(nd, box, ref, T)
    mc = syn.WATER_MC
    dr, nbins = 0.03, syn.n_bins_for(10.3, 0.03)
    g.track_histogram(dr, nbins)
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"], atom_frac=0.6, atom_disp=0.05)
    for s in range(2):
        g.mc_sweep(p, 40, s * 900, 900, stats=False)
        run = g.tracked_histogram().cpu().numpy().astype(np.uint64)
        moved = syn.Box("m", box.L, box.species, box.unit_offsets, g.coords_host(), 2)
        want, _ = orc.pair_histogram(moved, dr, nbins)
        assert np.array_equal(run, want)


def test_flexible_batched_matches_oracle(nd, orc):
    import torch
    T = syn.water_tables()
    mc = syn.WATER_MC
    boxes = [_distorted(300, 20.8, 50 + i) for i in range(3)]
    gb = [_gbox(nd, b, r, T) for b, r in boxes]
    E0 = [g.total_energy() for g in gb]
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"], atom_frac=0.5, atom_disp=0.05)
    batch = nd.Batch(gb)
    stats = batch.run(2, [p] * 3, [9, 10, 11], [0, 0, 0], trace=True)
    torch.cuda.synchronize()
    for i, ((box, ref), g) in enumerate(zip(boxes, gb)):
        r0 = orc.intra_reference(ref)
        tr = {k: v.cpu().numpy() for k, v in stats[i]["trace"].items()}
        xyz = box.xyz.copy()
        o = orc.mc_run_flex(box, T, xyz, mc["kT"], mc["max_disp"], mc["max_rot"], 0.5, 0.05, K_WATER, r0, 9 + i, 0,
                            2 * box.n_units, forced=tr["accepted"])
        assert np.all(np.abs(tr["dE"] - o["dE"]) <= 1e-6 * o["sabs"])
        assert not ((tr["accepted"] != o["acc"]) & (o["tie"] == 0)).any()
        assert f32_ulps(g.coords_host(), xyz, box.L).max() <= 2
        assert abs((stats[i]["E_total"] - E0[i]) - np.sum(o["dE"][o["acc"] == 1])) <= 1e-6 * np.sum(o["sabs"])
    batch.close()
