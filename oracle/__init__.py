"""Python access to the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark.  The library under test never imports
it, and it never imports the library.

Every function takes numpy arrays in the layouts documented in oracle.c and
returns numpy arrays.  Parity status of each function (what pins it) is
listed in oracle.c's header comments and in the test files.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = C.c_double
_i = C.c_int
_u64 = C.c_uint64
_i64 = C.c_int64
_p = C.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    sig = {
        "orc_abi_version": (_i, []),
        "orc_max_threads": (_i, []),
        "orc_set_threads": (None, [_i]),
        "orc_splitmix64": (_u64, [_u64, _u64]),
        "orc_uniform": (_d, [_u64, _u64, _i]),
        "orc_pair_index": (_i, [_i, _i, _i]),
        "orc_table_u": (_d, [_p, _i, _d, _d, _d]),
        "orc_table_du": (_d, [_p, _i, _d, _d, _d]),
        "orc_analytic_u": (_d, [_d, _d, _d, _d, _d, _d, _i]),
        "orc_total_energy": (None, [_i, _d, _i, _p, _p, _p, _p, _i, _d, _d, _p, _p]),
        "orc_delta_e": (None, [_i, _d, _i, _p, _p, _i, _p, _p, _p, _i, _d, _d, _p, _p]),
        "orc_propose": (_i, [_i, _d, _i, _p, _p, _d, _d, _i, _u64, _u64, _p]),
        "orc_mc_run": (_i64, [_i, _d, _i, _p, _i, _p, _p, _p, _i, _d, _d, _d, _d, _d, _i,
                              _u64, _u64, _i64, _d, _p, _p, _p, _p, _p, _p, _p]),
        "orc_intra_reference": (None, [_i, _d, _i, _p, _p, _p]),
        "orc_intra_energy": (None, [_i, _d, _i, _p, _i, _p, _p, _p, _p, _p, _p]),
        "orc_intra_forces": (None, [_i, _d, _i, _p, _i, _p, _p, _p, _p, _p]),
        "orc_propose_flex": (_i, [_i, _d, _i, _p, _p, _d, _d, _i, _d, _d, _u64, _u64, _p, _p, _p]),
        "orc_mc_run_flex": (_i64, [_i, _d, _i, _p, _i, _p, _p, _p, _i, _d, _d, _d, _d, _d, _i, _d, _d, _p,
                                   _p, _u64, _u64, _i64, _d, _p, _p, _p, _p, _p, _p, _p, _p]),
        "orc_edge2": (_d, [_i, _d]),
        "orc_r2": (_d, [_d, _d, _d, _d, _d, _d, _d]),
        "orc_pair_histogram": (None, [_i, _d, _i, _p, _p, _d, _i, _p, _p]),
        "orc_gr_normalize": (None, [_p, _i, _i, _d, _d, _p, _p]),
        "orc_sq": (None, [_p, _i, _i, _d, _d, _p, _d, _p, _i, _p]),
        "orc_hist_broad": (None, [_i, _d, _i, _p, _p, _d, _i, _d, _p]),
        "orc_hist_broad_backward": (None, [_i, _d, _i, _p, _p, _d, _i, _d, _p, _p]),
        "orc_sq_adjoint": (None, [_p, _i, _i, _d, _d, _d, _p, _p, _p, _i, _p]),
        "orc_forces": (None, [_i, _d, _i, _p, _p, _p, _p, _i, _d, _d, _p, _p]),
        "orc_hist_broad_backward_atoms": (None, [_i, _d, _i, _p, _p, _d, _i, _d, _p, _i, _p, _p]),
        "orc_forces_atoms": (None, [_i, _d, _i, _p, _p, _p, _p, _i, _d, _d, _i, _p, _p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def splitmix64(seed: int, i: int) -> int:
    return int(_load().orc_splitmix64(seed, i))


def uniform(seed: int, trial: int, draw: int) -> float:
    return float(_load().orc_uniform(seed, trial, draw))


def pair_index(a: int, b: int, m: int) -> int:
    return int(_load().orc_pair_index(a, b, m))


def table_u(row, h, r_cut, r) -> float:
    row = _c(row, np.float32)
    return float(_load().orc_table_u(_ptr(row), row.shape[0], h, r_cut, r))


def table_du(row, h, r_cut, r) -> float:
    row = _c(row, np.float32)
    return float(_load().orc_table_du(_ptr(row), row.shape[0], h, r_cut, r))


def analytic_u(r, sigma, eps, qq, kc, r_cut, shift_lj=True) -> float:
    return float(_load().orc_analytic_u(r, sigma, eps, qq, kc, r_cut, int(shift_lj)))


def unit_of_atom(unit_offsets) -> np.ndarray:
    counts = np.diff(np.asarray(unit_offsets))
    return np.repeat(np.arange(len(counts), dtype=np.int32), counts)


def total_energy(box, tables):
    xyz = _c(box.xyz, np.float32)
    sp = _c(box.species, np.uint8)
    uo = unit_of_atom(box.unit_offsets)
    U = _c(tables.U, np.float32)
    E = C.c_double()
    S = C.c_double()
    _load().orc_total_energy(box.n_atoms, box.L, box.n_species, _ptr(sp), _ptr(uo), _ptr(xyz),
                             _ptr(U), U.shape[1], tables.h, tables.r_cut, C.byref(E), C.byref(S))
    return E.value, S.value


def delta_e(box, tables, unit, newpos):
    xyz = _c(box.xyz, np.float32)
    sp = _c(box.species, np.uint8)
    uoff = _c(box.unit_offsets, np.int32)
    U = _c(tables.U, np.float32)
    npos = _c(newpos, np.float64)
    dE = C.c_double()
    S = C.c_double()
    _load().orc_delta_e(box.n_atoms, box.L, box.n_species, _ptr(sp), _ptr(uoff), int(unit),
                        _ptr(xyz), _ptr(npos), _ptr(U), U.shape[1], tables.h, tables.r_cut,
                        C.byref(dE), C.byref(S))
    return dE.value, S.value


def propose(box, xyz, max_disp, max_rot, order, seed, t):
    xyz = _c(xyz, np.float32)
    uoff = _c(box.unit_offsets, np.int32)
    out = np.zeros(64 * 3)
    u = _load().orc_propose(box.n_atoms, box.L, box.n_units, _ptr(uoff), _ptr(xyz),
                            max_disp, max_rot, int(order), seed, t, _ptr(out))
    na = int(uoff[u + 1] - uoff[u])
    return u, out[: 3 * na].reshape(na, 3)


def mc_run(box, tables, xyz, kT, max_disp, max_rot, seed, first_trial, n_trials,
           order=0, tie_rel=1e-6, forced=None, E_total=0.0):
    """Run the sequential Metropolis chain; xyz (float32 [3,N]) is updated in place."""
    assert xyz.dtype == np.float32 and xyz.flags.c_contiguous
    sp = _c(box.species, np.uint8)
    uoff = _c(box.unit_offsets, np.int32)
    U = _c(tables.U, np.float32)
    n = int(n_trials)
    dE = np.zeros(n)
    sabs = np.zeros(n)
    acc = np.zeros(n, np.uint8)
    tie = np.zeros(n, np.uint8)
    unit = np.zeros(n, np.int32)
    f = None if forced is None else _c(forced, np.uint8)
    Et = C.c_double(E_total)
    n_acc = _load().orc_mc_run(box.n_atoms, box.L, box.n_species, _ptr(sp), box.n_units,
                               _ptr(uoff), _ptr(xyz), _ptr(U), U.shape[1], tables.h,
                               tables.r_cut, kT, max_disp, max_rot, int(order), seed,
                               first_trial, n, tie_rel, _ptr(f), _ptr(dE), _ptr(sabs),
                               _ptr(acc), _ptr(tie), _ptr(unit), C.byref(Et))
    if n_acc < 0:
        raise ValueError("unit with more than 64 atoms")
    return dict(n_acc=int(n_acc), dE=dE, sabs=sabs, acc=acc, tie=tie, unit=unit, E_total=Et.value)


def intra_reference(box, xyz=None):
    """r0 of every intramolecular pair: float64 [N * 8] (atom a, partner slot b - first atom)."""
    xyz = _c(box.xyz if xyz is None else xyz, np.float32)
    uoff = _c(box.unit_offsets, np.int32)
    if np.diff(uoff).max() > 8:
        raise ValueError("intramolecular reference lengths take units of at most 8 atoms")
    r0 = np.zeros(box.n_atoms * 8)
    _load().orc_intra_reference(box.n_atoms, box.L, box.n_units, _ptr(uoff), _ptr(xyz), _ptr(r0))
    return r0


def intra_energy(box, kint, r0, xyz=None):
    """(intramolecular harmonic energy, sum of |terms|)."""
    xyz = _c(box.xyz if xyz is None else xyz, np.float32)
    sp = _c(box.species, np.uint8)
    uoff = _c(box.unit_offsets, np.int32)
    k = _c(kint, np.float64)
    r0 = _c(r0, np.float64)
    E = C.c_double()
    S = C.c_double()
    _load().orc_intra_energy(box.n_atoms, box.L, box.n_species, _ptr(sp), box.n_units, _ptr(uoff), _ptr(xyz),
                             _ptr(k), _ptr(r0), C.byref(E), C.byref(S))
    return E.value, S.value


def intra_forces(box, kint, r0, xyz=None):
    """Gradient of intra_energy: [3][N]."""
    xyz = _c(box.xyz if xyz is None else xyz, np.float32)
    sp = _c(box.species, np.uint8)
    uoff = _c(box.unit_offsets, np.int32)
    k = _c(kint, np.float64)
    r0 = _c(r0, np.float64)
    grad = np.zeros((3, box.n_atoms))
    _load().orc_intra_forces(box.n_atoms, box.L, box.n_species, _ptr(sp), box.n_units, _ptr(uoff), _ptr(xyz),
                             _ptr(k), _ptr(r0), _ptr(grad))
    return grad


def propose_flex(box, xyz, max_disp, max_rot, order, atom_frac, atom_disp, seed, t):
    """(unit, first moved atom, new positions [na, 3]) of trial t with single-atom moves."""
    xyz = _c(xyz, np.float32)
    uoff = _c(box.unit_offsets, np.int32)
    out = np.zeros(64 * 3)
    a0 = C.c_int()
    na = C.c_int()
    u = _load().orc_propose_flex(box.n_atoms, box.L, box.n_units, _ptr(uoff), _ptr(xyz), max_disp, max_rot,
                                 int(order), atom_frac, atom_disp, seed, t, _ptr(out), C.byref(a0), C.byref(na))
    return u, a0.value, out[: 3 * na.value].reshape(na.value, 3)


def mc_run_flex(box, tables, xyz, kT, max_disp, max_rot, atom_frac, atom_disp, kint, r0, seed, first_trial,
                n_trials, order=0, tie_rel=1e-6, forced=None, E_total=0.0):
    """The Metropolis chain with intramolecular harmonic terms and single-atom
    moves; xyz (float32 [3,N]) is updated in place."""
    assert xyz.dtype == np.float32 and xyz.flags.c_contiguous
    sp = _c(box.species, np.uint8)
    uoff = _c(box.unit_offsets, np.int32)
    U = _c(tables.U, np.float32)
    k = _c(kint, np.float64)
    r0 = _c(r0, np.float64)
    n = int(n_trials)
    dE = np.zeros(n)
    sabs = np.zeros(n)
    acc = np.zeros(n, np.uint8)
    tie = np.zeros(n, np.uint8)
    unit = np.zeros(n, np.int32)
    atom = np.zeros(n, np.int32)
    f = None if forced is None else _c(forced, np.uint8)
    Et = C.c_double(E_total)
    n_acc = _load().orc_mc_run_flex(box.n_atoms, box.L, box.n_species, _ptr(sp), box.n_units, _ptr(uoff), _ptr(xyz),
                                    _ptr(U), U.shape[1], tables.h, tables.r_cut, kT, max_disp, max_rot, int(order),
                                    atom_frac, atom_disp, _ptr(k), _ptr(r0), seed, first_trial, n, tie_rel, _ptr(f),
                                    _ptr(dE), _ptr(sabs), _ptr(acc), _ptr(tie), _ptr(unit), _ptr(atom), C.byref(Et))
    if n_acc < 0:
        raise ValueError("unit with more than 64 atoms")
    return dict(n_acc=int(n_acc), dE=dE, sabs=sabs, acc=acc, tie=tie, unit=unit, atom=atom, E_total=Et.value)


def edge2(k, dr) -> float:
    return float(_load().orc_edge2(int(k), dr))


def r2(pi, pj, L) -> float:
    return float(_load().orc_r2(*map(float, pi), *map(float, pj), L))


def pair_histogram(box_or_xyz, dr, nbins, L=None, species=None, n_species=None):
    if L is None:
        box = box_or_xyz
        xyz, L, species, n_species = box.xyz, box.L, box.species, box.n_species
    else:
        xyz = box_or_xyz
    xyz = _c(xyz, np.float32)
    sp = _c(species, np.uint8)
    P = n_species * (n_species + 1) // 2
    counts = np.zeros((P, nbins), np.uint64)
    n_out = np.zeros(P, np.uint64)
    _load().orc_pair_histogram(xyz.shape[1], float(L), n_species, _ptr(sp), _ptr(xyz), dr,
                               int(nbins), _ptr(counts), _ptr(n_out))
    return counts, n_out


def gr_normalize(counts, dr, V, npairs):
    c = _c(counts, np.float64)
    P, nb = c.shape
    g = np.zeros_like(c)
    npairs = _c(npairs, np.float64)
    _load().orc_gr_normalize(_ptr(c), P, nb, dr, V, _ptr(npairs), _ptr(g))
    return g


def sq(g, dr, rho, w, self_term, Q):
    g = _c(g, np.float64)
    P, nb = g.shape
    w = _c(w, np.float64)
    Q = _c(Q, np.float64)
    S = np.zeros(Q.shape[0])
    _load().orc_sq(_ptr(g), P, nb, dr, rho, _ptr(w), self_term, _ptr(Q), Q.shape[0], _ptr(S))
    return S


def hist_broad(box, dr, nbins, sigma, xyz=None):
    xyz = _c(box.xyz if xyz is None else xyz, np.float32)
    sp = _c(box.species, np.uint8)
    P = box.n_species * (box.n_species + 1) // 2
    out = np.zeros((P, nbins))
    _load().orc_hist_broad(box.n_atoms, box.L, box.n_species, _ptr(sp), _ptr(xyz), dr,
                           int(nbins), sigma, _ptr(out))
    return out


def hist_broad_backward(box, dr, nbins, sigma, A, xyz=None):
    xyz = _c(box.xyz if xyz is None else xyz, np.float32)
    sp = _c(box.species, np.uint8)
    A = _c(A, np.float64)
    grad = np.zeros((3, box.n_atoms))
    _load().orc_hist_broad_backward(box.n_atoms, box.L, box.n_species, _ptr(sp), _ptr(xyz), dr,
                                    int(nbins), sigma, _ptr(A), _ptr(grad))
    return grad


def hist_broad_backward_atoms(box, dr, nbins, sigma, A, sel, xyz=None):
    """hist_broad_backward for the atoms sel only (each a sum over all N
    partners): [3][len(sel)]."""
    xyz = _c(box.xyz if xyz is None else xyz, np.float32)
    sp = _c(box.species, np.uint8)
    A = _c(A, np.float64)
    sel = _c(sel, np.int32)
    grad = np.zeros((3, sel.shape[0]))
    _load().orc_hist_broad_backward_atoms(box.n_atoms, box.L, box.n_species, _ptr(sp), _ptr(xyz), dr,
                                          int(nbins), sigma, _ptr(A), sel.shape[0], _ptr(sel), _ptr(grad))
    return grad


def sq_adjoint(dLdS, nbins, dr, rho, V, w, npairs, Q):
    dLdS = _c(dLdS, np.float64)
    w = _c(w, np.float64)
    npairs = _c(npairs, np.float64)
    Q = _c(Q, np.float64)
    P = w.shape[0]
    A = np.zeros((P, nbins))
    _load().orc_sq_adjoint(_ptr(dLdS), P, int(nbins), dr, rho, V, _ptr(w), _ptr(npairs), _ptr(Q),
                           Q.shape[0], _ptr(A))
    return A


def forces(box, tables, xyz=None):
    xyz = _c(box.xyz if xyz is None else xyz, np.float32)
    sp = _c(box.species, np.uint8)
    uo = unit_of_atom(box.unit_offsets)
    U = _c(tables.U, np.float32)
    grad = np.zeros((3, box.n_atoms))
    E = C.c_double()
    _load().orc_forces(box.n_atoms, box.L, box.n_species, _ptr(sp), _ptr(uo), _ptr(xyz), _ptr(U),
                       U.shape[1], tables.h, tables.r_cut, _ptr(grad), C.byref(E))
    return grad, E.value


def forces_atoms(box, tables, sel, xyz=None):
    """The energy gradient of forces() for the atoms sel only: [3][len(sel)]."""
    xyz = _c(box.xyz if xyz is None else xyz, np.float32)
    sp = _c(box.species, np.uint8)
    uo = unit_of_atom(box.unit_offsets)
    U = _c(tables.U, np.float32)
    sel = _c(sel, np.int32)
    grad = np.zeros((3, sel.shape[0]))
    _load().orc_forces_atoms(box.n_atoms, box.L, box.n_species, _ptr(sp), _ptr(uo), _ptr(xyz), _ptr(U),
                             U.shape[1], tables.h, tables.r_cut, sel.shape[0], _ptr(sel), _ptr(grad))
    return grad


# ----------------------------------------------------------------------
# Derived quantities written out from Eq. 1's definitions (no library code).
# ----------------------------------------------------------------------
def pair_counts_total(species, n_species):
    """Npairs_p: N_a(N_a-1)/2 for like pairs, N_a N_b for unlike pairs."""
    n = np.bincount(np.asarray(species), minlength=n_species).astype(np.float64)
    out = []
    for a in range(n_species):
        for b in range(a, n_species):
            out.append(n[a] * (n[a] - 1) / 2 if a == b else n[a] * n[b])
    return np.array(out)


def eq1_weights(species, n_species, b):
    """Eq. 1 weights w_p = (2 - delta_ab) c_a c_b b_a b_b and the flat term sum c b^2."""
    n = np.bincount(np.asarray(species), minlength=n_species).astype(np.float64)
    c = n / n.sum()
    w = []
    for a in range(n_species):
        for bb in range(a, n_species):
            w.append((2.0 - (1.0 if a == bb else 0.0)) * c[a] * c[bb] * b[a] * b[bb])
    return np.array(w), float(np.sum(c * np.asarray(b) ** 2))
