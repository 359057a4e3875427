"""FP64 oracle of the empirical-potential (EMP) update of the refinement loop.

TEST INFRASTRUCTURE ONLY: imported by tests/ (and nothing the library
uses).  Plain numpy in the order of the method's steps; every function
names the passage it follows.  The library's own implementation (HIP
kernels behind nd_emp_update) shares no code with this file.

The method (Sec. "Algorithmic Principle"; Sec. "Correctness", Eq. 2): the
difference dS_i(Q) = S_exp,i(Q) - S_sim,i(Q) of each measured profile i is
fitted by a series of Poisson functions in Q space, the fit is turned into
the partial pair types through the inverse of the Eq. 1 weight matrix (a
pseudo-inverse of the matrix enlarged by a unit matrix when there are fewer
profiles than partials), and its real-space counterpart is added to the
potential as the EMP.

Readings (the paper prints no formula for the Poisson functions and Eq. 2
is garbled):
  * Poisson functions in r: p_n(r) = (r/s)^n exp(-r/s) / (4 pi rho s^3 (n+2)!),
    n = 1 .. n_terms, normalised so that 4 pi rho int r^2 p_n dr = 1.  Their
    Eq. 1-style transform 4 pi rho int r^2 p_n(r) sinc(Q r) dr has the closed
    form  P_n(Q) = sin((n+2) a) / ((n+2) Q s (1 + Q^2 s^2)^((n+2)/2)),
    a = atan(Q s), with P_n(0) = 1.
  * Fit: least squares over the Q grid, coefficients c_i from
    (G + ridge tr(G)/n_terms I) c_i = B^T dS_i with B[q, n] = P_n(Q_q) and
    G = B^T B.
  * Eq. 2 with w^-1: the partials' coefficients C_p = sum_i (W+)_{p i} c_i,
    W+ the inverse of the profiles-by-partials weight matrix W (w_ip of
    Eq. 1) when it is square, else the pseudo-inverse of W enlarged with
    id_weight times the unit matrix (rows of zero data).
  * Real space: the update dU_p(r) = -feedback kT sum_n C_pn p_n(r) (more
    correlation in the data than in the model lowers the potential there),
    shifted to zero at the cutoff like the reference potential and zero
    beyond; the EMP accumulates the updates, and if emp_max > 0 it is
    scaled down so that max |EMP| <= emp_max.
"""
from __future__ import annotations

import math

import numpy as np

from . import sq as _sq


def poisson_q(Q, sigma, n_terms):
    """P_n(Q), n = 1..n_terms: [n_terms][nQ] (closed form above)."""
    Q = np.asarray(Q, dtype=np.float64)
    out = np.empty((n_terms, Q.shape[0]))
    a = np.arctan(Q * sigma)
    base = 1.0 + (Q * sigma) ** 2
    for i, n in enumerate(range(1, n_terms + 1)):
        with np.errstate(invalid="ignore", divide="ignore"):
            v = np.sin((n + 2) * a) / ((n + 2) * Q * sigma * base ** ((n + 2) / 2.0))
        out[i] = np.where(Q == 0.0, 1.0, v)
    return out


def poisson_r(r, sigma, n_terms, rho):
    """p_n(r), n = 1..n_terms: [n_terms][len(r)]."""
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros((n_terms, r.shape[0]))
    pos = r > 0.0
    x = r[pos] / sigma
    for i, n in enumerate(range(1, n_terms + 1)):
        logv = n * np.log(x) - x - math.lgamma(n + 3) - math.log(4.0 * math.pi * rho * sigma ** 3)
        out[i, pos] = np.exp(logv)
    return out


def weight_pinv(W, id_weight=1.0):
    """W+ of Eq. 2: the inverse of W [n_prof][P] when square, otherwise the
    pseudo-inverse of W stacked over id_weight * I (P x P)."""
    W = np.asarray(W, dtype=np.float64)
    n_prof, P = W.shape
    if n_prof == P:
        return np.linalg.inv(W)
    Wa = np.vstack([W, id_weight * np.eye(P)])
    return np.linalg.pinv(Wa)[:, :n_prof]


def fit_coefficients(dS, Q, sigma, n_terms, ridge=0.0):
    """Least-squares Poisson coefficients of each row of dS [n_prof][nQ]."""
    B = poisson_q(Q, sigma, n_terms).T  # [nQ][n_terms]
    G = B.T @ B
    if ridge > 0.0:
        G = G + ridge * np.trace(G) / n_terms * np.eye(n_terms)
    rhs = B.T @ np.asarray(dS, dtype=np.float64).T  # [n_terms][n_prof]
    return np.linalg.solve(G, rhs).T  # [n_prof][n_terms]


def emp_update(g, dr, rho, W, self_terms, Q, S_exp, sigma, n_terms, feedback, kT, ridge, id_weight,
               h, n_pts, r_cut, emp_old=None, emp_max=0.0):
    """One EMP update.  g [P][nbins] (the model's g(r)); W [n_prof][P];
    self_terms [n_prof]; S_exp [n_prof][nQ].  Returns (EMP [P][n_pts] after
    the update, dS [n_prof][nQ], C [P][n_terms])."""
    W = np.asarray(W, dtype=np.float64)
    n_prof, P = W.shape
    # simulated profiles (Eq. 1) and their differences from the data
    S_sim = np.array([_sq(g, dr, rho, W[i], self_terms[i], Q) for i in range(n_prof)])
    dS = np.asarray(S_exp, dtype=np.float64) - S_sim
    # Poisson fit of each profile, then Eq. 2's inverse weights
    c = fit_coefficients(dS, Q, sigma, n_terms, ridge)
    C = weight_pinv(W, id_weight) @ c  # [P][n_terms]
    # real space, shifted to zero at the cutoff
    r = np.arange(n_pts, dtype=np.float64) * h
    pr = poisson_r(r, sigma, n_terms, rho)  # [n_terms][n_pts]
    pc = poisson_r(np.array([r_cut]), sigma, n_terms, rho)[:, 0]
    dU = np.empty((P, n_pts))
    for p in range(P):
        h_r = C[p] @ pr
        h_c = C[p] @ pc
        dU[p] = np.where(r < r_cut, -feedback * kT * (h_r - h_c), 0.0)
    emp = dU if emp_old is None else np.asarray(emp_old, dtype=np.float64) + dU
    if emp_max > 0.0:
        m = np.abs(emp).max()
        if m > emp_max:
            emp = emp * (emp_max / m)
    return emp, dS, C
