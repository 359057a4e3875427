"""Pins of the oracle's flexible molecules (intramolecular harmonic terms
between every two atoms of a unit, and single-atom moves besides whole-
molecule moves; Sec. "Correctness") against the mathematics:

* the energy change of every trial equals the difference of two full
  recomputes (intermolecular pair sum plus intramolecular energy);
* a single-atom move translates that atom by at most atom_disp per axis and
  leaves every other atom where it was; a whole-molecule move of a molecule
  in its reference geometry changes the intramolecular energy only by the
  rounding of the new positions to float32;
* a lone diatomic unit under its harmonic term alone samples r with density
  proportional to r^2 exp(-k (r - r0)^2 / kT) (chi^2 goodness of fit).
"""
import math

import numpy as np
from scipy import stats

import synthetic as syn

K_WATER = np.array([0.0, 2000.0, 600.0])  # O-O (none within a molecule), O-H, H-H; kJ/mol/A^2


def _distorted_water(n_mol, L, seed):
    box = syn.water_box(n_mol, L, seed, "flex water")
    rng = np.random.default_rng(seed)
    x = box.xyz.astype(np.float64) + rng.normal(scale=0.03, size=box.xyz.shape)
    box.xyz = np.ascontiguousarray((x - L * np.floor(x / L)).astype(np.float32))
    box.xyz[box.xyz >= L] = 0.0
    return box


def test_flexible_delta_e_equals_full_recompute(orc):
    ref = syn.water_box(300, 20.8, 1001, "flex water")
    r0 = orc.intra_reference(ref)
    box = _distorted_water(300, 20.8, 1001)
    T = syn.water_tables()
    E0 = orc.total_energy(box, T)[0] + orc.intra_energy(box, K_WATER, r0)[0]
    seen_atom = seen_mol = 0
    for t in range(40):
        u, a0, newpos = orc.propose_flex(box, box.xyz, 0.3, math.radians(10), 0, 0.5, 0.05, 17, t)
        moved = box.xyz.copy()
        for a in range(newpos.shape[0]):
            moved[:, a0 + a] = newpos[a].astype(np.float32)
        mbox = syn.Box("m", box.L, box.species, box.unit_offsets, moved, 2)
        E1 = orc.total_energy(mbox, T)[0] + orc.intra_energy(mbox, K_WATER, r0)[0]
        xyz = box.xyz.copy()
        res = orc.mc_run_flex(box, T, xyz, syn.WATER_MC["kT"], 0.3, math.radians(10), 0.5, 0.05, K_WATER, r0, 17,
                              t, 1)
        assert abs(res["dE"][0] - (E1 - E0)) <= 1e-10 * max(1.0, abs(E0)), (t, res["dE"][0], E1 - E0)
        if newpos.shape[0] == 1:
            seen_atom += 1
            assert res["atom"][0] == a0
            d = np.abs(moved.astype(np.float64) - box.xyz.astype(np.float64))
            d = np.minimum(d, box.L - d)
            assert d.max() <= 0.05 + 1e-5 and np.count_nonzero(d.sum(axis=0)) == 1
        else:
            seen_mol += 1
            assert res["atom"][0] == -1
    assert seen_atom > 5 and seen_mol > 5


def test_whole_molecule_moves_keep_the_reference_geometry(orc):
    box = syn.water_box(300, 20.8, 1001, "rigid start")
    r0 = orc.intra_reference(box)
    assert orc.intra_energy(box, K_WATER, r0)[0] == 0.0
    for t in range(30):
        u, a0, newpos = orc.propose_flex(box, box.xyz, 0.3, math.radians(10), 0, 0.0, 0.05, 3, t)
        assert newpos.shape[0] == 3
        moved = box.xyz.copy()
        moved[:, a0:a0 + 3] = newpos.T.astype(np.float32)
        E = orc.intra_energy(syn.Box("m", box.L, box.species, box.unit_offsets, moved, 2), K_WATER, r0)[0]
        # float32 rounding of ~20 A coordinates: about 1e-6 A per length
        assert E <= K_WATER.max() * 3 * (4e-6) ** 2


def test_lone_harmonic_pair_samples_its_boltzmann_density(orc):
    L, r0v, k, kT = 12.0, 1.5, 4.0, 2.4777
    xyz = np.array([[5.0, 5.0 + r0v], [5.0, 5.0], [5.0, 5.0]], dtype=np.float32)
    box = syn.Box("pair", L, np.array([0, 1], np.uint8), np.array([0, 2], np.int32), xyz, 2)
    T = syn.potential_table(2, 5.0, 0.01, [None, None], [0.0, 0.0])  # no intermolecular terms
    r0 = orc.intra_reference(box)
    kint = np.array([0.0, k, 0.0])
    x = box.xyz.copy()
    n = 300_000
    samples = []
    for first in range(0, n, 1000):
        orc.mc_run_flex(box, T, x, kT, 0.0, 0.0, 1.0, 0.4, kint, r0, 7, first, 1000)
        if first >= 20_000:
            d = x[:, 1].astype(np.float64) - x[:, 0].astype(np.float64)
            d -= L * np.round(d / L)
            samples.append(math.sqrt(float(d @ d)))
    r = np.array(samples)
    edges = np.linspace(0.3, 2.7, 13)
    obs, _ = np.histogram(r, edges)
    from scipy.integrate import quad
    w = [quad(lambda q: q * q * math.exp(-k * (q - r0v) ** 2 / kT), a, b)[0] for a, b in zip(edges[:-1], edges[1:])]
    exp_counts = np.array(w) / sum(w) * obs.sum()
    keep = exp_counts > 20
    chi2 = float(np.sum((obs[keep] - exp_counts[keep]) ** 2 / exp_counts[keep]))
    # samples every 1000 trials are close to independent; p > 1e-3
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-3, (chi2, obs, exp_counts)


def test_intra_forces_are_the_gradient(orc):
    ref = syn.water_box(40, 12.0, 5, "ref")
    r0 = orc.intra_reference(ref)
    box = _distorted_water(40, 12.0, 5)
    g = orc.intra_forces(box, K_WATER, r0)
    h = 1e-3
    rng = np.random.default_rng(2)
    for _ in range(20):
        i, c = int(rng.integers(0, box.n_atoms)), int(rng.integers(0, 3))
        xp, xm = box.xyz.copy(), box.xyz.copy()
        xp[c, i] = np.float32(xp[c, i] + h)
        xm[c, i] = np.float32(xm[c, i] - h)
        step = float(xp[c, i]) - float(xm[c, i])
        ep = orc.intra_energy(box, K_WATER, r0, xp)[0]
        em = orc.intra_energy(box, K_WATER, r0, xm)[0]
        # central difference of a quadratic-in-r energy: error O(h^2 k / r)
        assert abs((ep - em) / step - g[c, i]) <= 1e-3 * max(1.0, abs(g[c, i]))
    # no net force within a unit (Newton's third law)
    assert np.abs(g.sum(axis=1)).max() <= 1e-9 * np.abs(g).sum()
