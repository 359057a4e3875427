"""The differentiated form at full size: the 99,999-atom water box (C5).

* The pair gradient of the broadened histogram (nd_hist_broad_backward) for
  a seeded adjoint A, and the energy gradient (nd_forces), on 100 seeded
  atoms against the FP64 oracle, which sums each sampled atom's terms over
  all 99,998 partners.
* The broadened histogram of all pairs against the oracle's, stored.
* Central finite differences (h = 1e-4 A) of chi^2 against the target S(Q)
  of the bumped-potential run (stored), through the whole forward
  (broadened histogram -> g -> S(Q) -> chi^2), against the gradient from
  the backward, on 100 seeded atoms, one seeded axis each.  This holds
  at any size where the forward is smooth in the coordinates: a pair counts
  only while r < L/2, so chi^2 jumps when a pair crosses L/2 if that pair's
  window (r +- 6 sigma) reaches the binned range.  With bins to 49.8 A and
  L/2 = 49.85 A about a third of the atoms have such a partner within 1e-4 A
  of L/2; binning to 49.6 A keeps every window that reaches the range
  inside r < L/2, and chi^2 is then smooth.
"""
import os
import sys

import numpy as np
import pytest

import synthetic as syn

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
from make_golden import read_rows  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nd():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_1904_08756_amd as nd
    nd.lib()
    return nd


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.set_threads(oracle.max_threads())
    return oracle


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c5(nd):
    box, T, cfg = syn.config_c5()
    g = nd.Box.from_synthetic(box)
    g.set_tables(T.U, T.h, T.r_cut)
    rng = np.random.default_rng(cfg["fd_seed"])
    sel = np.sort(rng.choice(box.n_atoms, 100, replace=False)).astype(np.int32)
    axis = rng.integers(0, 3, sel.shape[0])
    return box, T, cfg, g, sel, axis


def test_broad_forward_full_box_matches_oracle(nd, c5):
    """The broadened histogram of all 4,999,850,001 pairs against the oracle's
    (stored by tests/golden/make_golden.py), per bin to 1e-6 of the bin's
    count (at least 1e-6 of one count)."""
    box, T, cfg, g, sel, _ = c5
    say("broadened forward, 99,999 atoms, all pairs")
    got = nd.hist_broad(g, cfg["dr"], cfg["nbins"], cfg["sigma"]).cpu().numpy()
    want = read_rows("c5_hist_broad.txt")
    assert got.shape == want.shape
    err = np.abs(got - want)
    say(f"max |diff| / max(count, 1) = {np.max(err / np.maximum(want, 1.0)):.3e}")
    assert np.all(err <= 1e-6 * np.maximum(want, 1.0)), float(np.max(err / np.maximum(want, 1.0)))


def test_broad_backward_full_box_sampled(nd, orc, c5):
    import torch
    box, T, cfg, g, sel, _ = c5
    dr, nb, sigma = cfg["dr"], cfg["nbins"], cfg["sigma"]
    say("broadened backward, 99,999 atoms, 100 sampled atoms")
    A = np.random.default_rng(cfg["target_seed"]).normal(size=(3, nb))
    got = nd.hist_broad_backward(g, dr, nb, sigma, torch.as_tensor(A, device="cuda")).cpu().numpy()[:, sel]
    want = orc.hist_broad_backward_atoms(box, dr, nb, sigma, A, sel)
    scale = np.abs(want).max()
    err = np.abs(got - want)
    # the same bound as on the small box: FP32 weights, FP64 sums
    assert np.all(err <= 1e-5 * scale + 1e-4 * np.abs(want)), float(np.max(err / scale))


def test_forces_full_box_sampled(nd, orc, c5):
    box, T, cfg, g, sel, _ = c5
    say("forces, 99,999 atoms, 100 sampled atoms")
    grad, _E = nd.forces(g)
    got = grad.cpu().numpy()[:, sel]
    want = orc.forces_atoms(box, T, sel)
    scale = np.abs(want).max()
    assert np.all(np.abs(got - want) <= 1e-9 * scale + 1e-9 * np.abs(want)), float(
        np.max(np.abs(got - want)) / scale)


def test_chi2_gradient_finite_differences_full_box(nd, c5):
    import torch
    box, T, cfg, g, sel, axis = c5
    dr, sigma = cfg["dr"], cfg["sigma"]
    nb = syn.n_bins_for(49.6, dr)
    assert nb * dr + 6 * sigma < box.L / 2
    Q = syn.q_grid(1000)
    b = syn.water_b(0.0)
    Qt = torch.as_tensor(Q, device="cuda")
    # the oracle's S(Q) of the bumped-potential run (seed 1006), from the
    # broadened g of that box; stored by tests/golden/make_golden.py
    target = torch.as_tensor(read_rows("c5_target_sq.txt")[0], device="cuda")
    assert target.shape[0] == Q.shape[0]
    x0 = box.xyz.astype(np.float32)
    x = torch.as_tensor(x0, device="cuda").clone().requires_grad_(True)
    say("chi^2 gradient, 99,999 atoms: forward + backward")
    c2 = nd.Chi2Fn.apply(x, g, dr, nb, sigma, Qt, target, b)
    c2.backward()
    grad = x.grad.cpu().numpy().astype(np.float64)
    h = 1e-4
    fd = np.zeros(sel.shape[0])
    gs = np.zeros(sel.shape[0])
    say("chi^2 central differences, 100 atoms")
    with torch.no_grad():
        for q, (i, c) in enumerate(zip(sel, axis)):
            xp = x0.copy()
            xm = x0.copy()
            xp[c, i] = np.float32(xp[c, i] + h)
            xm[c, i] = np.float32(xm[c, i] - h)
            step = float(xp[c, i]) - float(xm[c, i])
            cp = float(nd.Chi2Fn.apply(torch.as_tensor(xp, device="cuda"), g, dr, nb, sigma, Qt, target, b))
            cm = float(nd.Chi2Fn.apply(torch.as_tensor(xm, device="cuda"), g, dr, nb, sigma, Qt, target, b))
            fd[q] = (cp - cm) / step
            gs[q] = grad[c, i]
    scale = np.abs(gs).max()
    err = np.abs(fd - gs)
    say(f"max |fd - grad| / max |grad| = {err.max() / scale:.3e}")
    # P12: relative error 1e-3 (plus 1e-4 of the gradient scale for the
    # components near zero).  Pairs without the moved atom give identical
    # integer bin sums at x + h and x - h, so the difference carries only the
    # moved atom's ~1e5 pair weights, whose FP32 roundoff over 2h stays near
    # 1e-5 of the scale.  A wrong sign, a missing term or factor shows up at
    # order one.
    assert np.all(err <= 1e-3 * np.abs(gs) + 1e-4 * scale), float(np.max(err / scale))
    # translation invariance of chi^2: the gradient sums to zero over atoms
    assert abs(grad.sum(axis=1)).max() <= 1e-6 * np.abs(grad).sum(axis=1).max()
