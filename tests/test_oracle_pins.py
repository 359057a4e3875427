"""Pins for the FP64 oracle: closed forms, invariants, brute force, statistics.

None of these compares the oracle with itself: every expected value comes
from mathematics the paper's definitions fix (special values of the
potentials, conservation laws, exact expectations on a torus, closed-form
transforms, finite differences) or from a published test vector.
"""
import math
import os

import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- RNG
def test_splitmix64_published_outputs(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    for idx, val in rows:
        assert orc.splitmix64(0, int(idx)) == int(val, 16)


def test_uniform_is_the_top_53_bits_of_the_published_outputs(orc):
    # draws 0 and 1 of trial 0 with seed 0 are outputs 0 and 1 of the
    # generator started from state 0 (tests/golden/splitmix64_seed0.txt)
    for d, x in ((0, 0xE220A8397B1DCDAF), (1, 0x6E789E6AA1B965F4)):
        assert orc.uniform(0, 0, d) == (x >> 11) * 2.0 ** -53


def test_uniform_draws_are_uniform_and_distinct(orc):
    u = np.array([orc.uniform(1234, t, d) for t in range(2000) for d in range(8)])
    assert u.min() >= 0.0 and u.max() < 1.0
    # Kolmogorov-Smirnov against U(0,1)
    from scipy import stats
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    assert len(np.unique(u)) == len(u)


# ---------------------------------------------------------------- P1
def test_analytic_special_values(orc):
    sig, eps, rc = 3.166, 0.65, 10.0
    # Lennard-Jones is zero at sigma and -eps at its minimum 2^(1/6) sigma
    assert abs(orc.analytic_u(sig, sig, eps, 0.0, 0.0, rc, 0)) < 1e-12
    assert abs(orc.analytic_u(2 ** (1 / 6) * sig, sig, eps, 0.0, 0.0, rc, 0) + eps) < 1e-12
    # shifted Coulomb: k q q (1/r - 1/rc), at rc/2 equal to k q q / rc
    assert abs(orc.analytic_u(rc / 2, 1.0, 0.0, -2.0, 1389.35458, rc, 1)
               - 1389.35458 * -2.0 / rc) < 1e-12
    # zero from the cutoff on
    assert orc.analytic_u(rc, sig, eps, 1.0, 1389.35458, rc, 1) == 0.0
    assert orc.analytic_u(rc + 1, sig, eps, 1.0, 1389.35458, rc, 1) == 0.0


@pytest.mark.parametrize("which", ["water", "sio2"])
def test_tables_match_closed_form_and_lerp_bound(orc, which):
    if which == "water":
        T = syn.water_tables()
        params = {(0, 0): (3.166, 0.65, 0.8476 ** 2), (0, 1): (1.0, 0.0, -0.8476 * 0.4238),
                  (1, 1): (1.0, 0.0, 0.4238 ** 2)}
    else:
        T = syn.sio2_tables()
        params = {(0, 0): (0.76, 0.18, 4.0), (0, 1): (2.13, math.sqrt(0.18 * 0.65), -2.0),
                  (1, 1): (3.5, 0.65, 1.0)}
    rc, h = T.r_cut, T.h
    rng = np.random.default_rng(5)
    for p, ab in enumerate(syn.pair_type_list(2)):
        sig, eps, qq = params[ab]
        row = T.U[p]
        f = lambda r: orc.analytic_u(r, sig, eps, qq, syn.K_COULOMB, rc, 1)
        # grid points at r >= r_min hold the closed form rounded to float32
        for k in (50, 51, 100, 317, 700, T.n_pts - 2):
            r = k * h
            assert abs(row[k] - f(r)) <= 2 * np.spacing(np.float32(abs(f(r)))) + 1e-6
        assert row[-1] == 0.0
        # between grid points: |lerp - U| <= h^2/8 max|U''| (+ float32 rounding)
        for r in rng.uniform(1.2, rc - 0.02, 200):
            i0 = int(r / h)
            a, b = i0 * h, (i0 + 1) * h
            ts = np.linspace(a, b, 9)
            hh = 1e-4
            u2 = max(abs(f(t + hh) - 2 * f(t) + f(t - hh)) / hh ** 2 for t in ts)
            bound = h * h / 8 * u2 * 1.05 + 4 * np.spacing(np.float32(max(abs(f(a)), abs(f(b))) + 1e-3))
            assert abs(orc.table_u(row, h, rc, r) - f(r)) <= bound + 1e-9
        # continuity at the cutoff
        assert abs(orc.table_u(row, h, rc, rc - 1e-9)) < 1e-5
        assert orc.table_u(row, h, rc, rc) == 0.0


def _tiny_box(xyz, L, species, units, n_species=2):
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32))
    species = np.asarray(species, dtype=np.uint8)
    offs = np.asarray(units, dtype=np.int32)
    return syn.Box("tiny", float(L), species, offs, xyz, n_species)


def test_two_atom_energy_across_boundary(orc):
    T = syn.water_tables()
    L = 20.8
    # O at x=0.5 and O at x=L-0.5: nearest image 1.0 apart
    box = _tiny_box([[0.5, L - 0.5], [3.0, 3.0], [4.0, 4.0]], L, [0, 0], [0, 1, 2])
    E, S = orc.total_energy(box, T)
    dist = abs((0.5 - float(np.float32(L - 0.5))) + L)
    assert abs(dist - 1.0) < 1e-5
    assert abs(E - orc.table_u(T.U[0], T.h, T.r_cut, dist)) < 1e-9 * abs(E)
    assert abs(S - abs(E)) < 1e-9 * abs(E)
    # same unit: excluded
    box2 = _tiny_box(box.xyz, L, [0, 0], [0, 2])
    assert orc.total_energy(box2, T) == (0.0, 0.0)
    # beyond the cutoff: zero
    box3 = _tiny_box([[0.5, 10.6], [3.0, 3.0], [4.0, 4.0]], L, [0, 0], [0, 1, 2])
    assert orc.total_energy(box3, T)[0] == 0.0


# ---------------------------------------------------------------- P2
@pytest.mark.parametrize("cfg", ["c1", "c2cut"])
def test_delta_e_equals_full_recompute(orc, cfg):
    if cfg == "c1":
        box, T, _ = syn.config_c1()
    else:
        box = syn.water_box(1000, 99.7 * (1000 / 33333) ** (1 / 3), 1002, "cut")
        T = syn.water_tables()
    rng = np.random.default_rng(7)
    E0, S0 = orc.total_energy(box, T)
    for t in rng.integers(0, 10 ** 6, 6):
        u, newpos = orc.propose(box, box.xyz, 0.3, math.radians(10), 0, 99, int(t))
        dE, sabs = orc.delta_e(box, T, u, newpos)
        moved = box.xyz.copy()
        a0 = box.unit_offsets[u]
        for a in range(newpos.shape[0]):
            moved[:, a0 + a] = newpos[a].astype(np.float32)
        E1, S1 = orc.total_energy(syn.Box("m", box.L, box.species, box.unit_offsets, moved, 2), T)
        assert abs(dE - (E1 - E0)) <= 1e-12 * (S0 + S1) + 1e-12 * sabs
        assert sabs > 0


# ---------------------------------------------------------------- P3
def test_rigid_move_invariants(orc):
    box, T, mc = syn.config_c1()
    L = box.L
    for t in range(0, 3000, 97):
        u, newpos = orc.propose(box, box.xyz, mc["max_disp"], mc["max_rot"], 0, 5, t)
        assert u == t % box.n_units
        a0 = box.unit_offsets[u]
        old = box.xyz[:, a0:a0 + 3].T.astype(np.float64)

        def unwrap(p):
            return p[0] + ((p - p[0] + L / 2) % L - L / 2)
        po, pn = unwrap(old), unwrap(newpos)
        for P in (po, pn):
            assert abs(np.linalg.norm(P[1] - P[0]) - 1.0) < 2e-5
            assert abs(np.linalg.norm(P[2] - P[0]) - 1.0) < 2e-5
            assert abs(np.linalg.norm(P[2] - P[1]) - 2 * math.sin(math.radians(54.735))) < 2e-5
        tau = np.array([mc["max_disp"] * (2 * orc.uniform(5, t, c) - 1) for c in range(3)])
        shift = pn.mean(axis=0) - po.mean(axis=0)
        shift = (shift + L / 2) % L - L / 2
        assert np.allclose(shift, tau, atol=2e-5)
        # rotation angle of the body frame equals theta = max_rot (2 u5 - 1)
        th = mc["max_rot"] * (2 * orc.uniform(5, t, 5) - 1)
        a = (po - po.mean(0))
        b = (pn - pn.mean(0))
        # Kabsch: the proper rotation taking a onto b (reflection-corrected)
        U_, _, Vt = np.linalg.svd(a.T @ b)
        dsign = np.sign(np.linalg.det(Vt.T @ U_.T))
        R = Vt.T @ np.diag([1.0, 1.0, dsign]) @ U_.T
        assert np.allclose(a @ R.T, b, atol=2e-5)
        ang = math.acos(max(-1.0, min(1.0, (np.trace(R) - 1) / 2)))
        assert abs(ang - abs(th)) < 5e-4


def test_single_atom_move_is_translation(orc):
    box, T, mc = syn.config_c3()
    for t in (0, 1, 99998, 123456):
        u, newpos = orc.propose(box, box.xyz, 0.2, 0.0, 0, 3, t)
        tau = np.array([0.2 * (2 * orc.uniform(3, t, c) - 1) for c in range(3)])
        d = (newpos[0] - box.xyz[:, u] + box.L / 2) % box.L - box.L / 2
        assert np.allclose(d, tau, atol=1e-5)
        assert np.all(newpos[0] >= 0) and np.all(newpos[0] < box.L)


# ---------------------------------------------------------------- P4
def test_zero_potential_accepts_everything(orc):
    box, T, mc = syn.config_c1()
    Z = syn.Tables(np.zeros_like(T.U), T.h, T.r_cut)
    xyz = box.xyz.copy()
    res = orc.mc_run(box, Z, xyz, mc["kT"], 0.3, mc["max_rot"], 1, 0, 300)
    assert res["n_acc"] == 300
    assert np.all(res["dE"] == 0.0)


def test_metropolis_samples_boltzmann_distance(orc):
    """Two atoms on a torus: the minimum-image distance has density
    proportional to r^2 exp(-U(r)/kT) for r < L/2."""
    from scipy import stats
    L, rc, h, kT = 6.0, 3.0, 0.01, 2.5
    r = np.arange(int(rc / h) + 1) * h
    U = (2.0 * kT * np.exp(-((r - 1.6) ** 2) / 0.18) - 1.0 * kT * np.exp(-((r - 2.4) ** 2) / 0.05))
    U[-1] = 0.0
    row = U.astype(np.float32)
    T = syn.Tables(np.stack([row, row, row]), h, rc)
    box = _tiny_box([[1.0, 2.0], [1.0, 1.5], [1.0, 1.0]], L, [0, 0], [0, 1, 2])
    xyz = box.xyz.copy()
    samples = []
    seed, t = 42, 0
    for _ in range(4000):  # sample the configuration every 50 trials
        orc.mc_run(box, T, xyz, kT, 2.5, 0.0, seed, t, 50)
        t += 50
        samples.append(orc.r2(xyz[:, 0], xyz[:, 1], L))
    # moves of up to 2.5 A in a 6 A box decorrelate within 50 trials
    d = np.sqrt(np.array(samples))
    edges = np.linspace(0.0, rc, 11)
    obs, _ = np.histogram(d[d < rc], bins=edges)
    fine = np.linspace(0, rc, 30001)
    Uf = np.interp(fine, r, row.astype(np.float64))
    dens = fine ** 2 * np.exp(-Uf / kT)
    # outside rc up to the corner the density is r^2 x (cube-truncated shell); only test r < rc
    cum = np.concatenate([[0], np.cumsum((dens[1:] + dens[:-1]) / 2 * np.diff(fine))])
    p = np.diff(np.interp(edges, fine, cum))
    p = p / p.sum()
    exp = p * obs.sum()
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-3


# ---------------------------------------------------------------- P5/P6/P7
def test_histogram_count_conservation(orc):
    box, T, mc = syn.config_c1()
    counts, n_out = orc.pair_histogram(box, mc["dr"], mc["nbins"])
    npairs = orc.pair_counts_total(box.species, 2)
    assert np.array_equal(counts.sum(1) + n_out, npairs.astype(np.uint64))


def test_uniform_box_expected_counts(orc):
    """i.i.d. uniform atoms on a torus: n_p(k) ~ Binomial(Npairs_p, Vshell(k)/L^3)
    with pairwise-independent pair displacements, so the variance is exact."""
    from scipy import stats
    box = syn.atomic_box((3000, 6000), 40.0, 77, ("Si", "O"))
    dr = 0.1
    nb = syn.n_bins_for(20.0 - 1e-6, dr)
    counts, _ = orc.pair_histogram(box, dr, nb)
    npairs = orc.pair_counts_total(box.species, 2)
    k = np.arange(nb)
    q = 4 * np.pi / 3 * ((k + 1) ** 3 - k ** 3) * dr ** 3 / box.L ** 3
    z_all = []
    for p in range(3):
        e = npairs[p] * q
        v = npairs[p] * q * (1 - q)
        z = (counts[p].astype(np.float64) - e) / np.sqrt(v)
        z_all.append(z[e > 20])
    z = np.concatenate(z_all)
    assert np.max(np.abs(z)) < 6.0
    chi2 = float((z ** 2).sum())
    df = len(z)
    assert 1e-4 < stats.chi2.sf(chi2, df) < 1 - 1e-4


def test_rigid_water_intramolecular_peaks(orc):
    box, T, mc = syn.config_c1()
    counts, _ = orc.pair_histogram(box, mc["dr"], mc["nbins"])
    n_mol = box.n_units
    npairs = orc.pair_counts_total(box.species, 2)
    k = np.arange(mc["nbins"])
    q = 4 * np.pi / 3 * ((k + 1) ** 3 - k ** 3) * mc["dr"] ** 3 / box.L ** 3
    # O-H intramolecular: 2 per molecule in bin 33 = [0.99, 1.02)
    inter_oh = (npairs[1] - 2 * n_mol) * q[33]
    assert abs(counts[1, 33] - (2 * n_mol + inter_oh)) < 6 * math.sqrt(inter_oh) + 1
    # H-H intramolecular: 1 per molecule in bin 54 = [1.62, 1.65)
    inter_hh = (npairs[2] - n_mol) * q[54]
    assert abs(counts[2, 54] - (n_mol + inter_hh)) < 6 * math.sqrt(inter_hh) + 1
    # neighbours of those bins hold no intramolecular pairs
    assert counts[1, 32] < 2 * n_mol / 4 and counts[2, 53] < n_mol / 4


# ---------------------------------------------------------------- P8
def _brute_hist(xyz, L, species, M, dr, nbins):
    """27-image search: the smallest |x_j + n L - x_i| over n in {-1,0,1}^3."""
    N = xyz.shape[1]
    P = M * (M + 1) // 2
    out = np.zeros((P, nbins), np.int64)
    shifts = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]) * L
    x = xyz.astype(np.float64)
    near_edge = 0
    for i in range(N):
        for j in range(i + 1, N):
            d = (x[:, j] - x[:, i])[None, :] + shifts
            r2 = np.min(np.sum(d * d, axis=1))
            r = math.sqrt(r2)
            if r >= nbins * dr:
                continue
            k = int(math.floor(r / dr))
            if abs(r / dr - round(r / dr)) < 1e-9:
                near_edge += 1
            a, b = sorted((int(species[i]), int(species[j])))
            out[a * M - a * (a - 1) // 2 + (b - a), k] += 1
    return out, near_edge


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_histogram_brute_force_tiny_boxes(orc, seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 11))
    L = float(rng.uniform(3.0, 8.0))
    xyz = (rng.random((3, N)) * L).astype(np.float32)
    sp = rng.integers(0, 2, N).astype(np.uint8)
    dr = 0.07
    nb = syn.n_bins_for(L / 2 - 1e-6, dr)
    got, _ = orc.pair_histogram(xyz, dr, nb, L=L, species=sp, n_species=2)
    want, near = _brute_hist(xyz, L, sp, 2, dr, nb)
    assert near == 0
    assert np.array_equal(got.astype(np.int64), want)


def test_histogram_dyadic_edges_and_boundaries(orc):
    L = 4.0
    dr = 0.25
    nb = 7  # 1.75 < L/2
    cases = [
        # (xi, xj, expected bin or None)
        ((0.0, 0.0, 0.0), (0.75, 0.0, 0.0), 3),        # r^2 == edge2[3] exactly -> bin 3
        ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), 0),         # coincident atoms
        ((0.0, 0.0, 0.0), (float(np.nextafter(np.float32(4.0), np.float32(0))), 0.0, 0.0), 0),
        ((0.25, 0.0, 0.0), (3.5, 0.0, 0.0), 3),        # across the boundary: 0.75
        ((0.0, 0.0, 0.0), (1.75, 0.0, 0.0), None),     # r == edge[nbins]: not counted
        ((0.0, 0.0, 0.0), (2.0, 0.0, 0.0), None),      # r == L/2: not counted
        ((0.0, 0.0, 0.0), (0.5, 0.5, 0.0), 2),         # r^2 = 0.5 in [0.25, 0.5625)
    ]
    for xi, xj, want in cases:
        xyz = np.array([xi, xj], dtype=np.float32).T.copy()
        got, n_out = orc.pair_histogram(xyz, dr, nb, L=L, species=np.zeros(2, np.uint8), n_species=1)
        if want is None:
            assert got.sum() == 0 and n_out[0] == 1
        else:
            assert got[0, want] == 1 and got.sum() == 1, (xi, xj, got)


# ---------------------------------------------------------------- P9
def test_sq_flat_background_values(orc):
    # sum c b^2 for H2O, D2O and SiO2 from the scattering lengths
    sp_w = np.array([0, 1, 1], np.uint8)
    for x, want in ((0.0, 20.545017), (1.0, 40.893097), (0.25, 12.086024), (0.5, 12.657707),
                    (0.75, 22.260065), (0.64, 16.922448)):
        w, self_term = orc.eq1_weights(sp_w, 2, syn.water_b(x))
        assert abs(self_term - want) < 5e-6
    w, self_term = orc.eq1_weights(np.array([0, 1, 1], np.uint8), 2, syn.SIO2_B)
    assert abs(self_term - 28.187940) < 5e-6
    assert np.allclose(w, [1.912689, 10.700732, 14.966582], atol=5e-6)
    w0, _ = orc.eq1_weights(sp_w, 2, syn.water_b(0.0))
    w1, _ = orc.eq1_weights(sp_w, 2, syn.water_b(1.0))
    assert np.allclose(w0, [3.741645, -9.643296, 6.213387], atol=5e-6)
    assert np.allclose(w1, [3.741645, 17.205250, 19.778774], atol=5e-6)


def test_sq_of_ideal_gas_is_flat(orc):
    Q = syn.q_grid()
    g = np.ones((3, 500))
    S = orc.sq(g, 0.03, 0.1, [3.7, -9.6, 6.2], 20.545017, Q)
    assert np.all(S == 20.545017)


def test_sq_box_function_closed_form(orc):
    """g - 1 = 1 on [a, b]: the integral of r^2 sinc(Qr) is
    (1/Q) [sin(Qr)/Q^2 - r cos(Qr)/Q] from a to b."""
    dr, a, b, rho = 0.01, 2.0, 3.5, 0.1
    nb = 800
    g = np.ones((1, nb))
    r = (np.arange(nb) + 0.5) * dr
    g[0, (r > a) & (r < b)] = 2.0
    Q = np.array([0.5, 1.0, 2.5, 7.0, 15.0])
    S = orc.sq(g, dr, rho, [1.3], 0.0, Q)
    F = lambda q, x: (np.sin(q * x) / q ** 2 - x * np.cos(q * x) / q) / q
    exact = 1.3 * 4 * np.pi * rho * (F(Q, b) - F(Q, a))
    # midpoint-rule bound: (b-a) dr^2 / 24 max |d2/dr2 (r^2 sinc(Qr))|
    bound = 1.3 * 4 * np.pi * rho * (b - a) * dr ** 2 / 24 * (2 + 4 * Q * b + (Q * b) ** 2 / 1.0) / 1.0
    assert np.all(np.abs(S - exact) <= bound)
    # linear in the weights
    S2 = orc.sq(g, dr, rho, [2.6], 0.0, Q)
    assert np.allclose(S2, 2 * S, rtol=1e-14, atol=0)


def test_sq_large_q_tends_to_flat_term(orc):
    box, T, mc = syn.config_c1()
    counts, _ = orc.pair_histogram(box, mc["dr"], mc["nbins"])
    npairs = orc.pair_counts_total(box.species, 2)
    V = box.L ** 3
    g = orc.gr_normalize(counts, mc["dr"], V, npairs)
    w, self_term = orc.eq1_weights(box.species, 2, syn.water_b(0.0))
    Q = np.array([200.0, 400.0, 800.0])
    S = orc.sq(g, mc["dr"], box.n_atoms / V, w, self_term, Q)
    # oscillating tail decays like 1/Q around the flat term
    assert np.all(np.abs(S - self_term) < np.array([3.0, 1.5, 0.8]))


def test_gr_shell_volume_is_the_exact_shell_integral(orc):
    """g = n / (npairs Vshell / V) with Vshell(k) the volume between the
    spheres of radius k dr and (k + 1) dr: the integral of 4 pi r^2 over the
    bin, by adaptive quadrature.  The midpoint form 4 pi r_k^2 dr (3.6% off
    at k = 1) or the inner-edge form would fail this at any k."""
    from scipy.integrate import quad
    dr, nb = 0.03, 400
    for V, npairs, n in ((1.0, 1.0, 1.0), (7.25, 3.0, 5.0)):
        g = orc.gr_normalize(np.full((1, nb), n), dr, V, np.array([npairs]))
        shell = n * V / (npairs * g[0])
        exact = np.array([quad(lambda r: 4.0 * np.pi * r * r, k * dr, (k + 1) * dr, epsabs=0, epsrel=1e-13)[0]
                          for k in range(nb)])
        assert np.allclose(shell, exact, rtol=1e-12, atol=0.0)
    # the pin separates the plausible wrong forms from the right one
    k = np.arange(nb)
    midpoint = 4.0 * np.pi * ((k + 0.5) * dr) ** 2 * dr
    inner = 4.0 * np.pi * (k * dr) ** 2 * dr
    assert not np.allclose(midpoint, exact, rtol=1e-12, atol=0.0)
    assert not np.allclose(inner, exact, rtol=1e-12, atol=0.0)


def test_gr_of_uniform_box_is_one(orc):
    box = syn.atomic_box((4000, 4000), 30.0, 5, ("A", "B"))
    dr = 0.3
    nb = syn.n_bins_for(15.0 - 1e-6, dr)
    counts, _ = orc.pair_histogram(box, dr, nb)
    npairs = orc.pair_counts_total(box.species, 2)
    g = orc.gr_normalize(counts, dr, box.L ** 3, npairs)
    k = np.arange(nb)
    q = 4 * np.pi / 3 * ((k + 1) ** 3 - k ** 3) * dr ** 3 / box.L ** 3
    sd = np.sqrt((1 - q) / (npairs[:, None] * q))
    sel = q * npairs.min() > 50
    assert np.all(np.abs(g[:, sel] - 1.0) < 6 * sd[:, sel])


# ---------------------------------------------------------------- P11
def test_broadened_weights_sum_to_one(orc):
    sigma, dr, nb = 0.02, 0.03, 300
    L = 20.0
    for r in (0.5, 1.0, 3.333, 7.77, 8.0):
        box = _tiny_box([[1.0, 1.0 + r], [1.0, 1.0], [1.0, 1.0]], L, [0, 0], [0, 1, 2], 1)
        nh = orc.hist_broad(box, dr, nb, sigma)
        assert abs(nh.sum() - 1.0) < 1e-8
        # mass centred on the pair distance
        centre = ((np.arange(nb) + 0.5) * dr * nh[0]).sum()
        assert abs(centre - float(np.float32(1.0 + r) - np.float32(1.0))) < 1e-3


def test_broadened_tends_to_histogram(orc):
    box, T, mc = syn.config_c1()
    dr, nb = mc["dr"], mc["nbins"]
    counts, _ = orc.pair_histogram(box, dr, nb)
    nh = orc.hist_broad(box, dr, nb, 1e-5)
    # with sigma -> 0 every pair farther than 6 sigma from an edge counts fully
    assert np.abs(nh - counts).max() <= 2.0
    assert abs(nh.sum() - counts.sum()) <= 2.0


# ---------------------------------------------------------------- P12
def _energy_of(orc, box, T, xyz):
    return orc.total_energy(syn.Box("x", box.L, box.species, box.unit_offsets, xyz, box.n_species), T)[0]


def test_forces_finite_differences_and_newton(orc):
    box = syn.water_box(20, 12.0, 11)
    T = syn.water_tables(r_cut=6.0)
    grad, E = orc.forces(box, T)
    E0, _ = orc.total_energy(box, T)
    assert abs(E - E0) <= 1e-9 * max(1.0, abs(E0))
    # Newton's third law: the gradient sums to zero
    assert np.all(np.abs(grad.sum(axis=1)) <= 1e-7 * np.abs(grad).sum(axis=1))
    h = 1e-4
    uo = orc.unit_of_atom(box.unit_offsets)
    x = box.xyz.astype(np.float64)
    tested = 0
    for i in range(box.n_atoms):
        d = x - x[:, i:i + 1]
        d -= box.L * np.round(d / box.L)
        r = np.sqrt((d * d).sum(0))
        other = (uo != uo[i]) & (r < T.r_cut + 3 * h)
        # the interpolant is piecewise linear in r: skip atoms with a partner
        # whose distance lies within 3h of a table knot (slope jump)
        f = r[other] / T.h
        if np.any(np.minimum(f - np.floor(f), np.ceil(f) - f) < 3 * h / T.h):
            continue
        tested += 1
        for c in range(3):
            xp = box.xyz.copy(); xm = box.xyz.copy()
            xp[c, i] = np.float32(xp[c, i] + h)
            xm[c, i] = np.float32(xm[c, i] - h)
            step = float(xp[c, i]) - float(xm[c, i])
            # energy differences through the incremental form (exact zero for the
            # unit's unmoved atoms) avoid cancellation against a large total
            u = int(uo[i])
            a0 = int(box.unit_offsets[u]); a1 = int(box.unit_offsets[u + 1])
            dEp = orc.delta_e(box, T, u, xp[:, a0:a1].T.astype(np.float64))[0]
            dEm = orc.delta_e(box, T, u, xm[:, a0:a1].T.astype(np.float64))[0]
            fd = (dEp - dEm) / step
            assert abs(fd - grad[c, i]) <= 1e-5 * np.abs(grad[:, i]).sum() + 1e-6, (i, c, fd, grad[c, i])
        if tested >= 12:
            break
    assert tested >= 4


def _chi2_parts(orc, box, xyz, dr, nb, sigma, Q, target, b):
    nh = orc.hist_broad(box, dr, nb, sigma, xyz=xyz)
    npairs = orc.pair_counts_total(box.species, box.n_species)
    V = box.L ** 3
    g = orc.gr_normalize(nh, dr, V, npairs)
    w, self_term = orc.eq1_weights(box.species, box.n_species, b)
    S = orc.sq(g, dr, box.n_atoms / V, w, self_term, Q)
    return float(((S - target) ** 2).sum()), S, w, npairs, V


def test_chi2_gradient_finite_differences(orc):
    box = syn.water_box(40, 10.0, 12)
    sigma, dr = 0.02, 0.03
    nb = syn.n_bins_for(5.0 - 1e-6, dr)
    Q = syn.q_grid(200)
    b = syn.water_b(0.0)
    target = np.full(Q.shape, 20.0) + 0.5 * np.sin(Q)
    chi2, S, w, npairs, V = _chi2_parts(orc, box, box.xyz, dr, nb, sigma, Q, target, b)
    A = orc.sq_adjoint(2 * (S - target), nb, dr, box.n_atoms / V, V, w, npairs, Q)
    grad = orc.hist_broad_backward(box, dr, nb, sigma, A)
    assert np.all(np.abs(grad.sum(axis=1)) <= 1e-8 * np.abs(grad).sum(axis=1) + 1e-12)
    rng = np.random.default_rng(4)
    h = 1e-4
    for i in rng.integers(0, box.n_atoms, 6):
        for c in range(3):
            xp = box.xyz.copy(); xm = box.xyz.copy()
            xp[c, i] = np.float32(xp[c, i] + h)
            xm[c, i] = np.float32(xm[c, i] - h)
            step = float(xp[c, i]) - float(xm[c, i])
            fd = (_chi2_parts(orc, box, xp, dr, nb, sigma, Q, target, b)[0]
                  - _chi2_parts(orc, box, xm, dr, nb, sigma, Q, target, b)[0]) / step
            scale = np.abs(grad).max()
            assert abs(fd - grad[c, i]) <= 1e-3 * abs(grad[c, i]) + 1e-5 * scale, (i, c, fd, grad[c, i])


def test_subset_gradients_equal_full_rows(orc):
    """The per-atom forms used at full box size give exactly the rows of the
    full gradients (the same sum over partners, atom by atom)."""
    box = syn.water_box(60, 12.0, 13)
    T = syn.water_tables(r_cut=5.5)
    sigma, dr = 0.02, 0.03
    nb = syn.n_bins_for(6.0 - 1e-6, dr)
    rng = np.random.default_rng(14)
    A = rng.normal(size=(3, nb))
    sel = np.array([0, 7, 33, 90, 179, 5], np.int32)
    full = orc.hist_broad_backward(box, dr, nb, sigma, A)
    sub = orc.hist_broad_backward_atoms(box, dr, nb, sigma, A, sel)
    assert np.array_equal(sub, full[:, sel])
    fg, _ = orc.forces(box, T)
    fs = orc.forces_atoms(box, T, sel)
    assert np.array_equal(fs, fg[:, sel])


def test_sq_adjoint_is_transpose(orc):
    rng = np.random.default_rng(8)
    P, nb, dr, rho, V = 3, 120, 0.05, 0.1, 1000.0
    Q = syn.q_grid(50)
    w = rng.normal(size=P)
    npairs = rng.uniform(1e3, 1e4, P)
    n = rng.normal(size=(P, nb))
    y = rng.normal(size=Q.shape[0])
    # linear part of counts -> S: S(n) - S(0)
    S_n = orc.sq(orc.gr_normalize(n, dr, V, npairs), dr, rho, w, 0.0, Q)
    S_0 = orc.sq(orc.gr_normalize(np.zeros_like(n), dr, V, npairs), dr, rho, w, 0.0, Q)
    A = orc.sq_adjoint(y, nb, dr, rho, V, w, npairs, Q)
    lhs = float(y @ (S_n - S_0))
    rhs = float((A * n).sum())
    assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + abs(rhs))
