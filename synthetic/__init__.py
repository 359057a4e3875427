"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only *generates inputs*: atom positions, species, molecule
layouts, potential tables, Q grids and bin specifications.  It holds none
of the method's arithmetic (no pair sums, no histograms, no Metropolis
decisions, no S(Q) transform); both the library and the oracle receive
what it produces as plain arrays.

The experimental ISIS water / silica data the paper refines against
(Sec. "Performance Test", "Correctness") are not available, so the boxes
below stand in for them: rigid water with its H/D contrast variants and
amorphous SiO2 built as single-atom units, at the paper's scale of about
1e5 atoms (abstract; Table "tab_speed").

Conventions used by every consumer:
  * coordinates are float32, structure-of-arrays ``xyz[3, N]`` (x row,
    then y row, then z row), wrapped into [0, L);
  * ``species`` is uint8 per atom; ``unit_offsets`` is int32[n_units + 1]
    (CSR: the atoms of unit u are ``unit_offsets[u]:unit_offsets[u+1]``);
  * potential tables are float32 ``[P, n_pts]`` on the grid r_k = k*h,
    P = M(M+1)/2 pair types in the order (0,0),(0,1),...,(0,M-1),(1,1),...
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Coulomb constant e^2 N_A / (4 pi eps0) in kJ mol^-1 Angstrom e^-2.
K_COULOMB = 1389.35458
# Gas constant in kJ mol^-1 K^-1.
R_GAS = 8.3144626e-3

# Rigid water geometry: O-H 1.0 Angstrom, H-O-H 109.47 degrees.
WATER_OH = 1.0
WATER_HALF_ANGLE_DEG = 54.735

# Neutron scattering lengths in fm.
B_O = 5.803
B_H = -3.739
B_D = 6.671
B_SI = 4.149


@dataclass
class Box:
    """A periodic cubic box of atoms grouped into rigid units."""

    name: str
    L: float
    species: np.ndarray          # uint8 [N]
    unit_offsets: np.ndarray     # int32 [n_units + 1]
    xyz: np.ndarray              # float32 [3, N]
    n_species: int
    species_names: tuple = ()
    meta: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.species.shape[0])

    @property
    def n_units(self) -> int:
        return int(self.unit_offsets.shape[0] - 1)


@dataclass
class Tables:
    """Tabulated pair potentials U_p(r_k), r_k = k*h, k = 0..n_pts-1."""

    U: np.ndarray        # float32 [P, n_pts]
    h: float
    r_cut: float

    @property
    def n_pts(self) -> int:
        return int(self.U.shape[1])


def n_pair_types(m: int) -> int:
    return m * (m + 1) // 2


def pair_type_list(m: int):
    """Pair types (a, b), a <= b, in table-row order."""
    return [(a, b) for a in range(m) for b in range(a, m)]


def _wrap_f32(pos: np.ndarray, L: float) -> np.ndarray:
    """Wrap float64 positions into [0, L) and round to float32.

    A value that rounds up to L (or beyond) is set to 0, its periodic image.
    """
    w = pos - L * np.floor(pos / L)
    f = w.astype(np.float32)
    f[f.astype(np.float64) >= L] = np.float32(0.0)
    f[f < 0] = np.float32(0.0)
    return f


def water_body_frame() -> np.ndarray:
    """Rigid water atoms (O, H, H) relative to their unweighted centroid."""
    s = math.sin(math.radians(WATER_HALF_ANGLE_DEG)) * WATER_OH
    c = math.cos(math.radians(WATER_HALF_ANGLE_DEG)) * WATER_OH
    body = np.array([[0.0, 0.0, 0.0], [s, 0.0, c], [-s, 0.0, c]])
    return body - body.mean(axis=0)


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotation matrices from Shoemake's unit quaternions."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    qx = a * np.sin(2 * np.pi * u2)
    qy = a * np.cos(2 * np.pi * u2)
    qz = b * np.sin(2 * np.pi * u3)
    qw = b * np.cos(2 * np.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (qy * qy + qz * qz)
    R[:, 0, 1] = 2 * (qx * qy - qz * qw)
    R[:, 0, 2] = 2 * (qx * qz + qy * qw)
    R[:, 1, 0] = 2 * (qx * qy + qz * qw)
    R[:, 1, 1] = 1 - 2 * (qx * qx + qz * qz)
    R[:, 1, 2] = 2 * (qy * qz - qx * qw)
    R[:, 2, 0] = 2 * (qx * qz - qy * qw)
    R[:, 2, 1] = 2 * (qy * qz + qx * qw)
    R[:, 2, 2] = 1 - 2 * (qx * qx + qy * qy)
    return R


def water_box(n_mol: int, L: float, seed: int, name: str = "water") -> Box:
    """Rigid waters with uniform centroids and uniform random orientations.

    Atom order is molecule-major (O, H, H); species O=0, H=1.  There is no
    overlap rejection: the paper leaves the initial placement to the user.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cen = rng.random((n_mol, 3)) * L
    R = _random_rotations(rng, n_mol)
    body = water_body_frame()
    pos = cen[:, None, :] + np.einsum("mij,aj->mai", R, body)
    pos = pos.reshape(-1, 3)
    xyz = _wrap_f32(pos.T.copy(), L)
    species = np.tile(np.array([0, 1, 1], dtype=np.uint8), n_mol)
    offs = (np.arange(n_mol + 1, dtype=np.int64) * 3).astype(np.int32)
    return Box(name, float(L), species, offs, np.ascontiguousarray(xyz), 2,
               ("O", "H"), {"n_mol": n_mol, "seed": seed})


def atomic_box(counts, L: float, seed: int, names=(), name: str = "atomic") -> Box:
    """Single-atom units placed i.i.d. uniformly, species in blocks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(sum(counts))
    pos = rng.random((3, n)) * L
    xyz = _wrap_f32(pos, L)
    species = np.concatenate([np.full(c, s, dtype=np.uint8) for s, c in enumerate(counts)])
    offs = np.arange(n + 1, dtype=np.int32)
    return Box(name, float(L), species, offs, np.ascontiguousarray(xyz), len(counts),
               tuple(names), {"seed": seed})


def mixed_unit_box(n_units: int, L: float, seed: int, max_atoms: int = 4, n_species: int = 3,
                   name: str = "mixed") -> Box:
    """Rigid units of 1..max_atoms atoms (uniform), species uniform per atom.

    Each unit's atoms sit at random offsets of length 0.8-1.2 A around a
    uniform centre; atoms are wrapped into [0, L) one by one, so units
    straddle the box faces.  A stand-in for molecules of several sizes.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(1, max_atoms + 1, n_units)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    n = int(offs[-1])
    pos = np.empty((3, n))
    for u in range(n_units):
        c = rng.random(3) * L
        for a in range(offs[u], offs[u + 1]):
            v = rng.normal(size=3)
            v *= rng.uniform(0.8, 1.2) / np.linalg.norm(v)
            pos[:, a] = c + (v if a > offs[u] else 0.0)
    species = rng.integers(0, n_species, n).astype(np.uint8)
    xyz = _wrap_f32(pos, L)
    return Box(name, float(L), species, offs, np.ascontiguousarray(xyz), n_species, (), {"seed": seed})


def mixed_tables(r_cut: float = 8.0, h: float = 0.01) -> Tables:
    """Three species with LJ (3.0/0.5, 3.4/0.3, 2.5/0.8 A, kJ/mol), charges +0.5, -0.3, -0.2 e."""
    return potential_table(3, r_cut, h, [(3.0, 0.5), (3.4, 0.3), (2.5, 0.8)], [0.5, -0.3, -0.2])


def potential_table(m: int, r_cut: float, h: float, lj, charges, r_min: float = 0.5,
                    shift_lj: bool = True, emp=None) -> Tables:
    """Tabulate Lennard-Jones + truncated-shifted Coulomb (+ optional EMP).

    ``lj`` maps species -> (sigma, eps) or None; unlike species use
    Lorentz-Berthelot mixing.  ``charges`` is a per-species list in e.
    ``emp`` maps a pair type (a, b) to a callable U(r) in kJ/mol.
    Entries with r_k < r_min hold the value at r_min.  The reference
    potential is force-field input to the method, so it is built here.
    """
    n_t = int(round(r_cut / h))
    if abs(n_t * h - r_cut) > 1e-9:
        raise ValueError("r_cut must be a multiple of h")
    r = np.arange(n_t + 1, dtype=np.float64) * h
    rr = np.maximum(r, r_min)
    rows = []
    for a, b in pair_type_list(m):
        u = np.zeros_like(rr)
        la, lb = lj[a], lj[b]
        if la is not None and lb is not None:
            sig = 0.5 * (la[0] + lb[0])
            eps = math.sqrt(la[1] * lb[1])
            def ljf(x):
                sr6 = (sig / x) ** 6
                return 4.0 * eps * (sr6 * sr6 - sr6)
            u += ljf(rr) - (ljf(r_cut) if shift_lj else 0.0)
        qq = charges[a] * charges[b]
        if qq != 0.0:
            u += K_COULOMB * qq * (1.0 / rr - 1.0 / r_cut)
        if emp is not None and (a, b) in emp:
            u += emp[(a, b)](rr)
        u[-1] = 0.0
        rows.append(u)
    return Tables(np.ascontiguousarray(np.array(rows).astype(np.float32)), float(h), float(r_cut))


def water_tables(r_cut: float = 10.0, h: float = 0.01, emp=None) -> Tables:
    """SPC/E-like rigid water: LJ on O-O only, O -0.8476 e, H +0.4238 e."""
    return potential_table(2, r_cut, h, [(3.166, 0.65), None], [-0.8476, 0.4238], emp=emp)


def sio2_tables(r_cut: float = 12.0, h: float = 0.01) -> Tables:
    """Si (0.76 A, 0.18 kJ/mol) and O (3.5 A, 0.65 kJ/mol), Si +2 e, O -1 e."""
    return potential_table(2, r_cut, h, [(0.76, 0.18), (3.5, 0.65)], [2.0, -1.0])


def oo_bump_emp(amplitude: float = 0.5, centre: float = 2.8, width: float = 0.1):
    """A Gaussian empirical-potential bump on the O-O pair type."""
    return {(0, 0): lambda r: amplitude * np.exp(-((r - centre) ** 2) / (2 * width * width))}


def q_grid(n: int = 1000, q_min: float = 0.1, q_max: float = 30.0) -> np.ndarray:
    return q_min + np.arange(n, dtype=np.float64) * ((q_max - q_min) / (n - 1))


def n_bins_for(r_max: float, dr: float) -> int:
    return int(math.floor(r_max / dr + 1e-9))


def kT_at(temperature: float) -> float:
    return R_GAS * temperature


# Scattering-length sets.  Species order matches the boxes above.
def water_b(d_fraction: float = 0.0):
    """(b_O, b_H,eff) for a water sample with the given D fraction on H."""
    return (B_O, d_fraction * B_D + (1.0 - d_fraction) * B_H)


SIO2_B = (B_SI, B_O)

WATER_MC = {"kT": kT_at(298.0), "max_disp": 0.3, "max_rot": math.radians(10.0)}
SIO2_MC = {"kT": kT_at(298.0), "max_disp": 0.2, "max_rot": 0.0}

C4_D_FRACTIONS = (0.0, 0.25, 0.5, 0.75, 1.0, 0.64)


def config_c1():
    """Tiny water box: 300 waters, L = 20.8 A."""
    box = water_box(300, 20.8, 1001, "C1 tiny water")
    return box, water_tables(), dict(WATER_MC, seed=1001, n_trials=1000,
                                     dr=0.03, nbins=n_bins_for(10.4, 0.03))


def config_c2():
    """Large water box: 33,333 waters (99,999 atoms), L = 99.7 A."""
    box = water_box(33333, 99.7, 1002, "C2 large water")
    return box, water_tables(), dict(WATER_MC, seed=1002, n_trials=10 * 33333,
                                     dr=0.03, nbins=n_bins_for(49.8, 0.03))


def config_c3():
    """Amorphous SiO2: 33,333 Si + 66,666 O in L = 114.7 A."""
    box = atomic_box((33333, 66666), 114.7, 1003, ("Si", "O"), "C3 SiO2")
    return box, sio2_tables(), dict(SIO2_MC, seed=1003, n_trials=10 * 99999,
                                    dr=0.03, nbins=n_bins_for(114.7 / 2, 0.03))


def c4_sizes(seed: int = 1004, n_boxes: int = 64, lo: int = 500, hi: int = 20000):
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(n_boxes)
    return [int(round(math.exp(math.log(lo) + x * (math.log(hi) - math.log(lo))))) for x in u]


def config_c4(n_boxes: int = 64):
    """Batched form: water boxes of log-uniform size at 0.0334 molecules/A^3."""
    boxes = []
    for b, n_mol in enumerate(c4_sizes(n_boxes=n_boxes)):
        L = (n_mol / 0.0334) ** (1.0 / 3.0)
        box = water_box(n_mol, L, 1004000 + b, f"C4 box {b}")
        box.meta["d_fraction"] = C4_D_FRACTIONS[b % 6]
        box.meta["nbins"] = n_bins_for(L / 2, 0.03)
        boxes.append(box)
    rc = 10.0
    return boxes, water_tables(r_cut=rc), dict(WATER_MC, seed=1004, sweeps=5, dr=0.03)


def config_c5():
    """Differentiated form on the 99,999-atom water start (seed 1002)."""
    box = water_box(33333, 99.7, 1002, "C5 water (C2 start)")
    return box, water_tables(), dict(sigma=0.02, dr=0.03, nbins=n_bins_for(49.8, 0.03),
                                     fd_seed=1005, target_seed=1006)


def config_scale(n_mol: int, seed: int = 1007):
    """Scale-up water box: n_mol rigid waters at the C2 density (0.1009
    atoms/A^3, L = 99.7 A for 33,333 waters), the sizes of the paper's speed
    table (1.2e6 to 3e7 atoms); histogram bins as C2 (0.03 A to 49.8 A)."""
    L = 99.7 * (n_mol / 33333.0) ** (1.0 / 3.0)
    box = water_box(n_mol, L, seed, f"water {3 * n_mol} atoms")
    return box, water_tables(), dict(WATER_MC, seed=seed, dr=0.03, nbins=n_bins_for(49.8, 0.03))


def unit_of_atom(box: Box) -> np.ndarray:
    """Unit index of every atom (expanded CSR)."""
    counts = np.diff(box.unit_offsets)
    return np.repeat(np.arange(box.n_units, dtype=np.int32), counts)


def species_counts(box: Box) -> np.ndarray:
    return np.bincount(box.species, minlength=box.n_species)
