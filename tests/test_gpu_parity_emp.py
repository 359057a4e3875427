"""Empirical-potential update (nd_emp_update) against the FP64 oracle
(oracle/emp.py), and the refinement loop on a synthetic target.

Inputs are the oracle's: the model's g(r) is the oracle's g of the box, and
the "measured" profiles are the oracle's S(Q) of a box run by the oracle
with a 0.5 kJ/mol Gaussian O-O bump at 2.8 A added to the potential (three
H/D weightings for water; one profile for SiO2).  The library's EMP, fit
coefficients and profile differences must match the oracle's to 1e-8 of
their scale (both FP64; the fit's normal equations are solved by different
factorisations), its tables the float32 rounding of reference + EMP to one
unit in the last place.
"""
import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu

D_FRACTIONS = (0.0, 0.5, 1.0)


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


def _target(orc, box, T, mc, sweeps, seed, dr, nbins, profiles, bump=0.5):
    """The oracle's S(Q) of `box` after `sweeps` sweeps with the O-O bump."""
    Tb = syn.water_tables(r_cut=T.r_cut, emp=syn.oo_bump_emp(bump, 2.8, 0.1))
    xyz = box.xyz.copy()
    orc.mc_run(box, Tb, xyz, mc["kT"], mc["max_disp"], mc["max_rot"], seed, 0, sweeps * box.n_units)
    moved = syn.Box("target", box.L, box.species, box.unit_offsets, xyz, box.n_species)
    counts, _ = orc.pair_histogram(moved, dr, nbins)
    V = box.L ** 3
    g = orc.gr_normalize(counts.astype(np.float64), dr, V, orc.pair_counts_total(box.species, box.n_species))
    Q = syn.q_grid()
    W, st = [], []
    for b in profiles:
        w, s = orc.eq1_weights(box.species, box.n_species, b)
        W.append(w)
        st.append(s)
    W, st = np.array(W), np.array(st)
    S = np.array([orc.sq(g, dr, box.n_atoms / V, W[i], st[i], Q) for i in range(len(profiles))])
    return W, st, S, Q


def _model_g(orc, box, dr, nbins):
    counts, _ = orc.pair_histogram(box, dr, nbins)
    return orc.gr_normalize(counts.astype(np.float64), dr, box.L ** 3, orc.pair_counts_total(box.species,
                                                                                               box.n_species))


def _compare(nd, orc, box, T, W, st, S_exp, Q, g, dr, prm, kT, updates=2):
    import torch

    from oracle import emp as E
    gb = nd.Box.from_synthetic(box)
    gb.set_tables(T.U, T.h, T.r_cut)
    V, rho = gb.density()
    gd = torch.as_tensor(g, device="cuda")
    emp_o = None
    for u in range(updates):
        dS, emp, C = nd.emp_update(gb, prm, W, st, gd, dr, torch.as_tensor(Q, device="cuda"),
                                   torch.as_tensor(S_exp, device="cuda"))
        emp_o, dS_o, C_o = E.emp_update(g, dr, rho, W, st, Q, S_exp, prm.sigma, prm.n_terms, prm.feedback, kT,
                                        prm.ridge, prm.id_weight, T.h, T.n_pts, T.r_cut, emp_old=emp_o,
                                        emp_max=prm.emp_max)
        dS, emp, C = dS.cpu().numpy(), emp.cpu().numpy(), C.cpu().numpy()
        sd, se, sc = np.abs(dS_o).max(), np.abs(emp_o).max(), np.abs(C_o).max()
        say(f"update {u}: max|EMP| {se:.4g} kJ/mol; |dEMP|/scale {np.abs(emp - emp_o).max() / se:.2e}, "
            f"|dC|/scale {np.abs(C - C_o).max() / sc:.2e}")
        assert np.abs(dS - dS_o).max() <= 1e-10 * sd
        assert np.abs(C - C_o).max() <= 1e-8 * sc
        assert np.abs(emp - emp_o).max() <= 1e-8 * se
        tab = gb.tables()
        want = (T.U.astype(np.float64) + emp_o).astype(np.float32)
        ulps = np.abs(tab.view(np.int32).astype(np.int64) - want.view(np.int32).astype(np.int64))
        assert ulps.max() <= 1, ulps.max()
    gb.close()
    return emp_o


def test_emp_update_water_three_profiles(nd, orc):
    box, T, mc = syn.config_c1()
    dr = 0.03
    nbins = syn.n_bins_for(10.3, dr)
    profiles = [syn.water_b(x) for x in D_FRACTIONS]
    W, st, S_exp, Q = _target(orc, box, T, mc, 2, 606, dr, nbins, profiles)
    g = _model_g(orc, box, dr, nbins)
    prm = nd.EmpParams(kT=mc["kT"], sigma=0.3, n_terms=30, feedback=0.8, ridge=1e-6)
    emp = _compare(nd, orc, box, T, W, st, S_exp, Q, g, dr, prm, mc["kT"])
    assert np.abs(emp).max() > 0.0


def test_emp_update_sio2_one_profile_and_cap(nd, orc):
    box = syn.atomic_box((400, 800), 23.0, 77, ("Si", "O"), "SiO2 small")
    T = syn.sio2_tables(r_cut=11.0)
    dr = 0.03
    nbins = syn.n_bins_for(11.3, dr)
    rng = np.random.default_rng(8)
    # "measured": the model's S(Q) plus a smooth low-Q feature (input only)
    g = _model_g(orc, box, dr, nbins)
    W = np.array([orc.eq1_weights(box.species, 2, syn.SIO2_B)[0]])
    st = np.array([orc.eq1_weights(box.species, 2, syn.SIO2_B)[1]])
    Q = syn.q_grid()
    S_sim = orc.sq(g, dr, box.n_atoms / box.L ** 3, W[0], st[0], Q)
    S_exp = (S_sim + 0.3 * np.exp(-(Q - 2.0) ** 2 / 0.5) * (1 + 0.1 * rng.normal(size=Q.shape[0])))[None, :]
    prm = nd.EmpParams(kT=syn.SIO2_MC["kT"], sigma=0.25, n_terms=24, feedback=1.0, ridge=1e-6, id_weight=1.0)
    _compare(nd, orc, box, T, W, st, S_exp, Q, g, dr, prm, syn.SIO2_MC["kT"])
    prm.emp_max = 0.05
    emp = _compare(nd, orc, box, T, W, st, S_exp, Q, g, dr, prm, syn.SIO2_MC["kT"], updates=1)
    assert abs(np.abs(emp).max() - 0.05) < 1e-12


def test_emp_update_rejects_bad_input(nd):
    import torch
    box, T, mc = syn.config_c1()
    gb = nd.Box.from_synthetic(box)
    gb.set_tables(T.U, T.h, T.r_cut)
    g = torch.ones((3, 100), dtype=torch.float64, device="cuda")
    Q = torch.as_tensor(syn.q_grid(), device="cuda")
    S = torch.zeros((3, Q.shape[0]), dtype=torch.float64, device="cuda")
    W = np.ones((3, 3))  # singular
    with pytest.raises(nd.NeudaError, match="INVALID"):
        nd.emp_update(gb, nd.EmpParams(kT=2.5), W, np.zeros(3), g, 0.03, Q, S)
    with pytest.raises(nd.NeudaError, match="INVALID"):
        nd.emp_update(gb, nd.EmpParams(kT=2.5, n_terms=100), np.eye(3), np.zeros(3), g, 0.03, Q, S)
    gb.close()


@pytest.mark.timeout(600)
def test_refinement_loop_reduces_the_misfit(nd, orc):
    """Empirical-potential Monte Carlo on a Lennard-Jones liquid of 2,000
    atoms (one profile, one pair type; it equilibrates within a few sweeps,
    so the misfit measures the potential and not the equilibration) towards
    the oracle's S(Q) of the same liquid with a 2 kJ/mol Gaussian bump at
    4.2 A added to its potential: the chi^2 after four EMP updates is well
    below its value before the first."""
    import oracle
    oracle.set_threads(oracle.max_threads())
    L, n = 46.4, 2000
    T = syn.potential_table(1, 12.0, 0.01, [(3.4, 1.0)], [0.0])
    Tb = syn.potential_table(1, 12.0, 0.01, [(3.4, 1.0)], [0.0],
                             emp={(0, 0): lambda r: 2.0 * np.exp(-(r - 4.2) ** 2 / (2 * 0.15 ** 2))})
    kT = syn.kT_at(120.0)
    dr = 0.03
    nbins = syn.n_bins_for(15.0, dr)
    box = syn.atomic_box((n,), L, 4242, ("Ar",), "LJ liquid")
    tbox = syn.atomic_box((n,), L, 4343, ("Ar",), "LJ target")
    say("oracle target: 2000 LJ atoms, 40 sweeps with the bump")
    x = tbox.xyz.copy()
    oracle.mc_run(tbox, Tb, x, kT, 0.5, 0.0, 4343, 0, 40 * n)
    moved = syn.Box("t", L, tbox.species, tbox.unit_offsets, x, 1)
    counts, _ = oracle.pair_histogram(moved, dr, nbins)
    g_t = oracle.gr_normalize(counts.astype(np.float64), dr, L ** 3, oracle.pair_counts_total(tbox.species, 1))
    W = np.array([[1.0]])
    st = np.array([1.0])
    Q = syn.q_grid()
    S_exp = oracle.sq(g_t, dr, n / L ** 3, W[0], 1.0, Q)[None, :]
    gb = nd.Box.from_synthetic(box)
    gb.set_tables(T.U, T.h, T.r_cut)
    p = nd.MCParams(kT, 0.5, 0.0)
    gb.mc_sweep(p, 5, 0, 40 * n, stats=False)  # equilibrate with the reference potential
    prm = nd.EmpParams(kT=kT, sigma=0.25, n_terms=40, feedback=0.6, ridge=1e-6, emp_max=3.0)
    hist, _ = nd.refine(gb, p, 5, W, st, S_exp, Q, dr, nbins, prm, iterations=5, sweeps=12, sample_sweeps=10,
                        first_trial=40 * n)
    tot = [sum(h) for h in hist]
    say("chi^2 per iteration:", ", ".join(f"{x:.4g}" for x in tot))
    assert tot[-1] < 0.5 * tot[0]
    gb.close()
