"""Pins of the oracle's empirical-potential update (oracle/emp.py) against
the mathematics, with no implementation to compare with:

* the closed-form Q-space Poisson functions equal the numerical Eq. 1-style
  transform of the real-space ones, and both are normalised to 1 at Q = 0;
* the least-squares fit recovers the coefficients of a difference built
  from the basis itself;
* the weight inverse: W W+ = I for three H/D water profiles; the Moore-
  Penrose conditions for one SiO2 profile enlarged by the unit matrix;
* the whole update: a measured profile set built as the model's S(Q) plus
  the Eq. 1 transform of known Poisson coefficients gives back exactly the
  potential -feedback kT sum C p_n (shifted at the cutoff); equal profiles
  give no update; more structure in the data lowers the potential there.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import synthetic as syn
from oracle import emp as E


def test_poisson_q_closed_form_equals_transform():
    rho, sigma = 0.1, 0.3
    for n in (1, 4, 12, 30):
        def p_n(r):
            return E.poisson_r(np.array([r]), sigma, n, rho)[n - 1, 0]
        # normalisation: 4 pi rho int r^2 p_n dr = 1
        norm = quad(lambda r: 4 * math.pi * rho * r * r * p_n(r), 0, 200 * sigma + 20, limit=400)[0]
        assert abs(norm - 1.0) < 1e-9
        for Q in (0.05, 0.7, 2.3, 9.0):
            # oscillatory quadrature (QAWO) of f(r) sin(Q r)
            val = quad(lambda r: 4 * math.pi * rho * r * p_n(r) / Q, 0, 200 * sigma + 20, weight="sin", wvar=Q,
                       limit=800)[0]
            closed = E.poisson_q(np.array([Q]), sigma, n)[n - 1, 0]
            assert abs(val - closed) <= 1e-9 * max(1.0, abs(closed)), (n, Q, val, closed)
    # Q = 0 and the approach to it
    assert np.all(E.poisson_q(np.array([0.0]), sigma, 10)[:, 0] == 1.0)
    assert np.all(np.abs(E.poisson_q(np.array([1e-6]), sigma, 10)[:, 0] - 1.0) < 1e-9)


def test_fit_recovers_basis_coefficients():
    """Six terms (Gram condition ~3e7): the coefficients themselves; thirty
    terms with a small ridge (the Gram matrix of overlapping Poisson
    functions is near singular there): the fitted difference."""
    Q = syn.q_grid()
    rng = np.random.default_rng(4)
    sigma, nt = 0.3, 6
    c_true = rng.normal(size=(2, nt))
    dS = c_true @ E.poisson_q(Q, sigma, nt)
    c = E.fit_coefficients(dS, Q, sigma, nt, ridge=0.0)
    assert np.allclose(c, c_true, rtol=1e-7, atol=1e-7 * np.abs(c_true).max())
    nt = 30
    B = E.poisson_q(Q, sigma, nt)
    c_true = rng.normal(size=(2, nt))
    dS = c_true @ B
    c = E.fit_coefficients(dS, Q, sigma, nt, ridge=1e-9)
    assert np.abs(c @ B - dS).max() <= 1e-4 * np.abs(dS).max()


def test_weight_inverse_square_and_enlarged():
    box, _, _ = syn.config_c1()
    import oracle
    W = np.array([oracle.eq1_weights(box.species, 2, syn.water_b(x))[0] for x in (0.0, 0.5, 1.0)])
    Wp = E.weight_pinv(W)
    assert np.allclose(W @ Wp, np.eye(3), atol=1e-12) and np.allclose(Wp @ W, np.eye(3), atol=1e-12)
    # one SiO2 profile: pseudo-inverse of [W; I]
    w1 = np.array([[1.912689, 10.700732, 14.966582]])
    Wa = np.vstack([w1, np.eye(3)])
    X = np.linalg.pinv(Wa)
    for a, b in ((Wa @ X @ Wa, Wa), (X @ Wa @ X, X)):
        assert np.allclose(a, b, atol=1e-12)
    assert np.allclose((Wa @ X).T, Wa @ X, atol=1e-12) and np.allclose((X @ Wa).T, X @ Wa, atol=1e-12)
    assert np.allclose(E.weight_pinv(w1), X[:, :1], atol=1e-14)


def _model(nb=300, dr=0.03):
    # a smooth model g(r) of three partials (input only)
    r = (np.arange(nb) + 0.5) * dr
    g = np.vstack([1.0 + 0.3 * np.exp(-(r - 2.8 + 0.1 * k) ** 2 / 0.08) * np.sin(3 * r) for k in range(3)])
    return g, dr


@pytest.mark.parametrize("n_prof", [3, 1])
def test_update_returns_the_potential_of_a_known_difference(n_prof):
    import oracle
    box, T, mc = syn.config_c1()
    g, dr = _model()
    rho = box.n_atoms / box.L ** 3
    Q = syn.q_grid()
    if n_prof == 3:
        W = np.array([oracle.eq1_weights(box.species, 2, syn.water_b(x))[0] for x in (0.0, 0.5, 1.0)])
    else:
        W = np.array([oracle.eq1_weights(box.species, 2, syn.water_b(0.0))[0]])
    st = np.full(n_prof, 10.0)
    sigma, nt, kT, fb = 0.3, 6, 2.4777, 0.7
    rng = np.random.default_rng(6)
    C_true = rng.normal(size=(3, nt))
    S_sim = np.array([oracle.sq(g, dr, rho, W[i], st[i], Q) for i in range(n_prof)])
    S_exp = S_sim + W @ (C_true @ E.poisson_q(Q, sigma, nt))
    h, n_pts, rc = T.h, T.n_pts, T.r_cut
    idw = 1.0 if n_prof == 3 else 1e-4
    emp, dS, C = E.emp_update(g, dr, rho, W, st, Q, S_exp, sigma, nt, fb, kT, 0.0, idw, h, n_pts, rc)
    r = np.arange(n_pts) * h
    pr = E.poisson_r(r, sigma, nt, rho)
    pc = E.poisson_r(np.array([rc]), sigma, nt, rho)[:, 0]
    if n_prof == 3:
        assert np.allclose(C, C_true, rtol=1e-6, atol=1e-6 * np.abs(C_true).max())
        want = np.where(r < rc, -fb * kT * (C_true @ pr - (C_true @ pc)[:, None]), 0.0)
        assert np.allclose(emp, want, rtol=1e-6, atol=1e-6 * np.abs(want).max())
    else:
        # fewer profiles than partials, unit rows of small weight: the update
        # reproduces the profile difference the data asks for, with the
        # least norm (it lies in the span of the weights)
        assert np.allclose(W @ C, W @ C_true, rtol=1e-5, atol=1e-5 * np.abs(W @ C_true).max())
        least = W.T @ np.linalg.solve(W @ W.T, W @ C_true)
        assert np.allclose(C, least, rtol=1e-5, atol=1e-5 * np.abs(least).max())
    assert emp[:, -1].max() == 0.0 and emp[:, -1].min() == 0.0  # zero at the cutoff
    # equal profiles: no update
    emp0, dS0, C0 = E.emp_update(g, dr, rho, W, st, Q, S_sim, sigma, nt, fb, kT, 0.0, 1.0, h, n_pts, rc)
    assert np.abs(emp0).max() < 1e-10 and np.abs(dS0).max() == 0.0


def test_more_structure_in_the_data_lowers_the_potential():
    import oracle
    box, T, mc = syn.config_c1()
    g, dr = _model()
    rho = box.n_atoms / box.L ** 3
    Q = syn.q_grid()
    W = np.array([oracle.eq1_weights(box.species, 2, syn.water_b(x))[0] for x in (0.0, 0.5, 1.0)])
    st = np.full(3, 10.0)
    # data: the model with an extra O-O peak at 3 A (added to g before Eq. 1)
    r = (np.arange(g.shape[1]) + 0.5) * dr
    g_exp = g.copy()
    g_exp[0] += 0.5 * np.exp(-(r - 3.0) ** 2 / (2 * 0.15 ** 2))
    S_exp = np.array([oracle.sq(g_exp, dr, rho, W[i], st[i], Q) for i in range(3)])
    emp, _, _ = E.emp_update(g, dr, rho, W, st, Q, S_exp, 0.2, 40, 1.0, 2.4777, 1e-8, 1.0, T.h, T.n_pts, T.r_cut)
    k3 = int(round(3.0 / T.h))
    assert emp[0, k3] < 0.0 and abs(emp[0, k3]) > 5 * max(abs(emp[1, k3]), abs(emp[2, k3]))
    # the cap scales the whole EMP
    capped, _, _ = E.emp_update(g, dr, rho, W, st, Q, S_exp, 0.2, 40, 1.0, 2.4777, 1e-8, 1.0, T.h, T.n_pts,
                                T.r_cut, emp_max=0.1)
    assert abs(np.abs(capped).max() - 0.1) < 1e-12
    assert np.allclose(capped, emp * (0.1 / np.abs(emp).max()))
