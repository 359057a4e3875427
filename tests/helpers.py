"""Small shared checks for the parity tests (no computation of the method)."""
import numpy as np


def f32_ulps(got, want, L):
    """Distance in float32 units in the last place between coordinates in
    [0, L) (both non-negative, so the bit patterns order like the values);
    an atom that wrapped on one side only counts by its periodic distance."""
    a = np.asarray(got, dtype=np.float32).view(np.int32).astype(np.int64)
    b = np.asarray(want, dtype=np.float32).view(np.int32).astype(np.int64)
    ulps = np.abs(a - b)
    d = np.abs(np.asarray(got, dtype=np.float64) - np.asarray(want, dtype=np.float64))
    wrapped = d > L / 2
    ulps[wrapped] = np.ceil((L - d[wrapped]) / np.spacing(np.float32(L))).astype(np.int64)
    return ulps


def expected_near_ties(dE, sabs, kT, tie_rel=1e-6):
    """Expected number of decisions whose threshold -kT ln u (u uniform,
    so the threshold is exponential with mean kT) falls within
    tie_rel * sabs of dE."""
    tau = tie_rel * np.asarray(sabs)
    dE = np.asarray(dE)
    return float(np.sum(np.exp(-np.maximum(dE - tau, 0.0) / kT) - np.exp(-np.maximum(dE + tau, 0.0) / kT)))
