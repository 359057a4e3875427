"""Python binding of the MI355X pair-sum library (include/neuda.h).

Thin ctypes layer: it marshals arguments to the C ABI and allocates device
outputs with torch; every step of the computation runs in the HIP kernels
of libneuda.so.  There is no CPU fallback: if the library is missing or no
GPU is present, the calls raise.

Method: Ma et al., "NeuDATool" (arXiv 1904.08756) -- the Metropolis pair sum
of Sec. "Algorithmic Flow" III, the N(r) histogram of Sec. "Acceleration
method", and Eq. 1.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np

__all__ = [
    "lib", "build", "Box", "MCParams", "pair_histogram", "gr_normalize", "sq_transform",
    "sq_adjoint", "hist_broad", "hist_broad_backward", "forces", "Chi2Fn", "EnergyFn",
    "chi2", "gr_normalize_f64", "pair_counts_total", "eq1_weights", "Batch",
    "ND_HOST", "ND_DEVICE", "NeudaError",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libneuda.so")

ND_HOST = 0
ND_DEVICE = 1
ND_ORDER_SEQ = 0
ND_ORDER_RANDOM = 1
ND_SCAN_CELLS = 0
ND_SCAN_FULL = 1
PROF = {"mc_scan": 0, "mc_corr": 1, "mc_decide": 2, "mc_propose": 3, "pair_hist": 4,
        "hist_broad": 5, "hist_broad_bwd": 6, "forces": 7}
STATUS = {0: "ND_OK", -1: "ND_E_INVALID", -2: "ND_E_RANGE", -3: "ND_E_OOM", -4: "ND_E_HIP",
          -5: "ND_E_STATE", -6: "ND_E_UNSUPPORTED"}


class NeudaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class nd_box_desc(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("n_species", C.c_int32), ("L", C.c_double),
                ("species", C.c_void_p), ("n_units", C.c_int32), ("unit_offsets", C.c_void_p),
                ("xyz", C.c_void_p), ("device", C.c_int32), ("stream", C.c_void_p)]


class nd_mc_params(C.Structure):
    _fields_ = [("kT", C.c_double), ("max_disp", C.c_double), ("max_rot", C.c_double),
                ("order", C.c_int32), ("k_batch", C.c_int32), ("tie_rel", C.c_double),
                ("scan", C.c_int32), ("atom_frac", C.c_double), ("atom_disp", C.c_double)]


class nd_mc_stats(C.Structure):
    _fields_ = [("trials", C.c_int64), ("accepted", C.c_int64), ("near_ties", C.c_int64),
                ("E_total", C.c_double), ("dE_sum", C.c_double)]


class nd_mc_trace(C.Structure):
    _fields_ = [("dE", C.c_void_p), ("sabs", C.c_void_p), ("accepted", C.c_void_p),
                ("unit", C.c_void_p)]


class nd_batch_plan(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("mc", C.c_void_p), ("seed", C.c_void_p),
                ("first_trial", C.c_void_p), ("dr", C.c_double), ("nbins", C.c_void_p),
                ("w", C.c_void_p), ("self_term", C.c_void_p), ("Q", C.c_void_p), ("nQ", C.c_int32),
                ("counts", C.c_void_p), ("g", C.c_void_p), ("S", C.c_void_p),
                ("trace", C.c_void_p)]


class nd_tuning(C.Structure):
    _fields_ = [("kind", C.c_int32), ("scan_waves", C.c_int32), ("n_max", C.c_int64),
                ("batch_target", C.c_double), ("hist_blocks_per_cu", C.c_int32), ("pad", C.c_int32)]


class nd_emp_params(C.Structure):
    _fields_ = [("sigma", C.c_double), ("n_terms", C.c_int32), ("pad", C.c_int32), ("feedback", C.c_double),
                ("kT", C.c_double), ("ridge", C.c_double), ("id_weight", C.c_double), ("emp_max", C.c_double)]


ND_TUNE_BOX = 0
ND_TUNE_BATCH = 1
TUNE_KINDS = {"box": ND_TUNE_BOX, "batch": ND_TUNE_BATCH}
# tuned launch parameters for this GPU, written by autotune.py
TUNING_FILE = os.path.join(_HERE, "tuning.txt")

EXPORTS = {
    "nd_abi_version": (C.c_int32, []),
    "nd_last_error": (C.c_char_p, []),
    "nd_box_create": (C.c_int32, [C.POINTER(nd_box_desc), C.POINTER(C.c_void_p)]),
    "nd_box_destroy": (C.c_int32, [C.c_void_p]),
    "nd_box_set_stream": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "nd_box_set_coords": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32]),
    "nd_box_get_coords": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32]),
    "nd_box_set_tables": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.c_double]),
    "nd_box_total_energy": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double)]),
    "nd_box_set_intra": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "nd_box_energy": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double)]),
    "nd_mc_sweep": (C.c_int32, [C.c_void_p, C.POINTER(nd_mc_params), C.c_uint64, C.c_uint64,
                                C.c_int64, C.POINTER(nd_mc_stats), C.POINTER(nd_mc_trace)]),
    "nd_pair_histogram": (C.c_int32, [C.c_void_p, C.c_double, C.c_int32, C.c_void_p, C.c_int32]),
    "nd_gr_normalize": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                    C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "nd_sq_transform": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                    C.c_void_p, C.c_double, C.c_void_p, C.c_int32, C.c_void_p,
                                    C.c_int32, C.c_void_p]),
    "nd_hist_broad": (C.c_int32, [C.c_void_p, C.c_double, C.c_int32, C.c_double, C.c_void_p,
                                  C.c_int32]),
    "nd_sq_adjoint": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                  C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                  C.c_void_p, C.c_int32, C.c_void_p]),
    "nd_hist_broad_backward": (C.c_int32, [C.c_void_p, C.c_double, C.c_int32, C.c_double,
                                           C.c_void_p, C.c_void_p, C.c_int32]),
    "nd_forces": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_int32]),
    "nd_forces_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "nd_gr_normalize_f64": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                        C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "nd_box_pair_counts": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "nd_box_density": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "nd_box_track_histogram": (C.c_int32, [C.c_void_p, C.c_double, C.c_int32]),
    "nd_box_tracked_histogram": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32]),
    "nd_box_accumulate": (C.c_int32, [C.c_void_p]),
    "nd_box_accumulated": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.c_int32]),
    "nd_box_set_profiling": (C.c_int32, [C.c_void_p, C.c_int32]),
    "nd_box_set_profiling_mask": (C.c_int32, [C.c_void_p, C.c_uint32]),
    "nd_box_profile": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double)]),
    "nd_box_count_scan": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "nd_eq1_weights": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "nd_chi2": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                            C.c_void_p]),
    "nd_box_save": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]),
    "nd_box_load": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "nd_batch_create": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "nd_batch_destroy": (C.c_int32, [C.c_void_p]),
    "nd_batch_run": (C.c_int32, [C.c_void_p, C.POINTER(nd_batch_plan), C.c_void_p]),
    "nd_batch_info": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "nd_emp_update": (C.c_int32, [C.c_void_p, C.POINTER(nd_emp_params), C.c_int32, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_int32, C.c_double, C.c_void_p, C.c_int32, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p]),
    "nd_box_get_tables": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32]),
    "nd_set_tuning": (C.c_int32, [C.c_void_p, C.c_int32]),
    "nd_get_tuning": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    "nd_load_tuning": (C.c_int32, [C.c_char_p]),
}

_lib = None

# Live handles, released at interpreter exit (batches before boxes) while
# the HIP runtime is still up, instead of from __del__ during teardown.
_live_batches = weakref.WeakSet()
_live_boxes = weakref.WeakSet()


def _release_all():
    for t in list(_live_batches):
        try:
            t.close()
        except Exception:
            pass
    for b in list(_live_boxes):
        try:
            b.close()
        except Exception:
            pass


_exit_hook = False


def _register_exit():
    # registered at the first handle, after torch has set up the GPU, so it
    # runs before anything torch registered earlier (atexit is last-in,
    # first-out)
    global _exit_hook
    if not _exit_hook:
        atexit.register(_release_all)
        _exit_hook = True


def build() -> str:
    from . import buildlib
    return buildlib.build()


def lib():
    """The loaded libneuda.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1904_08756_amd.build()")
    L = C.CDLL(LIB_PATH)
    missing = []
    for name, (res, args) in EXPORTS.items():
        try:
            f = getattr(L, name)
        except AttributeError:
            # a library built from other sources than this binding: the
            # entry point raises when called (tests check every export)
            missing.append(name)
            continue
        f.restype = res
        f.argtypes = args
    if "nd_box_create" in missing or "nd_last_error" in missing:
        raise ImportError(f"{LIB_PATH} does not export the neuda ABI")
    _lib = L
    if os.path.exists(TUNING_FILE) and not os.environ.get("NEUDA_NO_TUNING"):
        _check(L.nd_load_tuning(TUNING_FILE.encode()))
    return L


def set_tuning(entries):
    """Replace the library's tuning table: entries are dicts with kind
    ("box" or "batch"), n_max, scan_waves, batch_target, hist_blocks_per_cu."""
    arr = (nd_tuning * max(1, len(entries)))()
    for i, e in enumerate(entries):
        arr[i] = nd_tuning(TUNE_KINDS[e["kind"]], int(e.get("scan_waves", 0)), int(e["n_max"]),
                           float(e.get("batch_target", 0.0)), int(e.get("hist_blocks_per_cu", 0)), 0)
    _check(lib().nd_set_tuning(arr, len(entries)))


def get_tuning():
    """The library's tuning table as a list of dicts."""
    n = C.c_int32()
    _check(lib().nd_get_tuning(None, 0, C.byref(n)))
    arr = (nd_tuning * max(1, n.value))()
    _check(lib().nd_get_tuning(arr, n.value, C.byref(n)))
    names = {v: k for k, v in TUNE_KINDS.items()}
    return [dict(kind=names[x.kind], n_max=x.n_max, scan_waves=x.scan_waves, batch_target=x.batch_target,
                 hist_blocks_per_cu=x.hist_blocks_per_cu) for x in arr[:n.value]]


def tuning_for(kind, n_atoms):
    """The tuning entry the library applies to `kind` and n_atoms, or None."""
    for e in get_tuning():
        if e["kind"] == kind and n_atoms <= e["n_max"]:
            return e
    return None


def load_tuning(path):
    _check(lib().nd_load_tuning(os.fsencode(path)))


def _check(code):
    if code != 0:
        raise NeudaError(code, lib().nd_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the neuda library needs a HIP GPU; none is visible")
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def _host_f64(a, n=None):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and arr.shape[0] != n:
        raise ValueError("length mismatch")
    return arr


@dataclass
class MCParams:
    kT: float
    max_disp: float
    max_rot: float = 0.0
    order: int = ND_ORDER_SEQ
    k_batch: int = 0
    tie_rel: float = 0.0
    scan: int = ND_SCAN_CELLS
    atom_frac: float = 0.0
    atom_disp: float = 0.0

    def c(self):
        return nd_mc_params(self.kT, self.max_disp, self.max_rot, self.order, self.k_batch,
                            self.tie_rel, self.scan, self.atom_frac, self.atom_disp)


class Box:
    """A periodic box on one GPU (owns the device state of nd_box)."""

    def __init__(self, xyz, species, unit_offsets, L, n_species, device=0):
        torch = _torch()
        xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32))
        species = np.ascontiguousarray(np.asarray(species, dtype=np.uint8))
        offs = np.ascontiguousarray(np.asarray(unit_offsets, dtype=np.int32))
        if xyz.ndim != 2 or xyz.shape[0] != 3:
            raise ValueError("xyz must be [3, N]")
        self.N = int(xyz.shape[1])
        self.M = int(n_species)
        self.P = self.M * (self.M + 1) // 2
        self.L = float(L)
        self.n_units = int(offs.shape[0] - 1)
        self.species = species
        self.unit_offsets = offs
        self.device = int(device)
        torch.cuda.set_device(self.device)
        d = nd_box_desc(self.N, self.M, self.L, species.ctypes.data, self.n_units, offs.ctypes.data,
                        xyz.ctypes.data, self.device, _stream())
        h = C.c_void_p()
        _check(lib().nd_box_create(C.byref(d), C.byref(h)))
        self._h = h
        # changes whenever the coordinates change (set_coords, sweeps, load,
        # batch runs), so a saved autograd context can tell it is stale
        self.version = 0
        _live_boxes.add(self)
        _register_exit()

    @classmethod
    def from_synthetic(cls, sbox, device=0):
        return cls(sbox.xyz, sbox.species, sbox.unit_offsets, sbox.L, sbox.n_species, device)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("box destroyed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().nd_box_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        _check(lib().nd_box_set_stream(self.handle, _stream()))

    # -- measurement
    def set_profiling(self, enable: bool, kernels=None):
        """Event pairs around every profiled launch (kernels: names of PROF to
        restrict them to; the others launch without events)."""
        self._sync_stream()
        if kernels is None:
            _check(lib().nd_box_set_profiling(self.handle, int(enable)))
        else:
            mask = 0
            for k in kernels:
                mask |= 1 << PROF[k]
            _check(lib().nd_box_set_profiling_mask(self.handle, mask if enable else 0))

    def count_scan(self, enable: bool):
        """(candidates, survivors) the cell scan tested since the last call;
        then restarts counting (enable) or stops it."""
        self._sync_stream()
        c = C.c_int64()
        v = C.c_int64()
        _check(lib().nd_box_count_scan(self.handle, int(enable), C.byref(c), C.byref(v)))
        return c.value, v.value

    def profile(self, kernel: str):
        """(launches, total milliseconds) recorded for a kernel since profiling was enabled."""
        n = C.c_int64()
        ms = C.c_double()
        _check(lib().nd_box_profile(self.handle, PROF[kernel], C.byref(n), C.byref(ms)))
        return n.value, ms.value

    # -- state
    def set_tables(self, U, h, r_cut):
        U = np.ascontiguousarray(np.asarray(U, dtype=np.float32))
        if U.shape[0] != self.P:
            raise ValueError("table rows must equal the number of pair types")
        self._sync_stream()
        _check(lib().nd_box_set_tables(self.handle, U.ctypes.data, U.shape[1], float(h), float(r_cut)))
        self._n_pts = int(U.shape[1])
        self.version += 1

    def set_intra(self, k):
        """Intramolecular harmonic terms k_p (r - r0)^2 between every two atoms of a
        unit, r0 from the current coordinates (k: [P] kJ/mol/A^2, None removes them)."""
        self._sync_stream()
        if k is None:
            _check(lib().nd_box_set_intra(self.handle, None))
        else:
            kk = _host_f64(k, self.P)
            _check(lib().nd_box_set_intra(self.handle, kk.ctypes.data))

    def set_coords(self, xyz, keep_energy=False):
        torch = _torch()
        self._sync_stream()
        self.version += 1
        if isinstance(xyz, torch.Tensor) and xyz.is_cuda:
            t = xyz.detach().to(torch.float32).contiguous()
            _check(lib().nd_box_set_coords(self.handle, _dptr(t), ND_DEVICE, int(keep_energy)))
        else:
            a = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32))
            _check(lib().nd_box_set_coords(self.handle, a.ctypes.data, ND_HOST, int(keep_energy)))

    def coords(self):
        """Current coordinates as a float32 [3, N] device tensor."""
        torch = _torch()
        self._sync_stream()
        out = torch.empty((3, self.N), dtype=torch.float32, device=f"cuda:{self.device}")
        _check(lib().nd_box_get_coords(self.handle, _dptr(out), ND_DEVICE))
        return out

    def coords_host(self):
        out = np.empty((3, self.N), np.float32)
        self._sync_stream()
        _check(lib().nd_box_get_coords(self.handle, out.ctypes.data, ND_HOST))
        return out

    def save(self) -> bytes:
        """Checkpoint image of the box's Metropolis state (nd_box_save)."""
        self._sync_stream()
        n = C.c_size_t()
        _check(lib().nd_box_save(self.handle, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(lib().nd_box_save(self.handle, buf, C.byref(n)))
        return buf.raw[:n.value]

    def load(self, image: bytes):
        """Restore a checkpoint made by save() (nd_box_load)."""
        self._sync_stream()
        self.version += 1
        buf = C.create_string_buffer(bytes(image), len(image))
        _check(lib().nd_box_load(self.handle, buf, len(image)))

    # -- running histogram and its accumulation
    def track_histogram(self, dr, nbins):
        """Keep a running N(r) updated by every accepted move (nbins = 0 stops)."""
        self._sync_stream()
        _check(lib().nd_box_track_histogram(self.handle, float(dr), int(nbins)))
        self._track_nbins = int(nbins)

    def tracked_histogram(self):
        """The running counts as an int64 [P, nbins] device tensor (uint64 values)."""
        torch = _torch()
        self._sync_stream()
        out = torch.empty((self.P, self._track_nbins), dtype=torch.int64, device=f"cuda:{self.device}")
        _check(lib().nd_box_tracked_histogram(self.handle, _dptr(out), ND_DEVICE))
        return out

    def accumulate(self):
        """Add the running counts to the sum of samples."""
        self._sync_stream()
        _check(lib().nd_box_accumulate(self.handle))

    def accumulated(self):
        """(mean counts [P, nbins] float64 device tensor, number of samples)."""
        torch = _torch()
        self._sync_stream()
        out = torch.empty((self.P, self._track_nbins), dtype=torch.float64, device=f"cuda:{self.device}")
        n = C.c_int64()
        _check(lib().nd_box_accumulated(self.handle, _dptr(out), C.byref(n), ND_DEVICE))
        return out, n.value

    def tables(self):
        """The tables the energy kernels use (reference + EMP), float32 [P, n_pts] host array."""
        self._sync_stream()
        out = np.empty((self.P, self._n_pts), np.float32)
        _check(lib().nd_box_get_tables(self.handle, out.ctypes.data, ND_HOST))
        return out

    def density(self):
        """(V, rho): box volume and number density (nd_box_density)."""
        V = C.c_double()
        rho = C.c_double()
        _check(lib().nd_box_density(self.handle, C.byref(V), C.byref(rho)))
        return V.value, rho.value

    def total_energy(self):
        E = C.c_double()
        self._sync_stream()
        _check(lib().nd_box_total_energy(self.handle, C.byref(E)))
        return E.value

    def energy(self):
        E = C.c_double()
        self._sync_stream()
        _check(lib().nd_box_energy(self.handle, C.byref(E)))
        return E.value

    # -- method
    def mc_sweep(self, params: MCParams, seed: int, first_trial: int, n_trials: int,
                 trace: bool = False, stats: bool = True):
        torch = _torch()
        self._sync_stream()
        tr = None
        tr_t = None
        if trace:
            dev = f"cuda:{self.device}"
            tr_t = dict(dE=torch.empty(n_trials, dtype=torch.float64, device=dev),
                        sabs=torch.empty(n_trials, dtype=torch.float64, device=dev),
                        accepted=torch.empty(n_trials, dtype=torch.uint8, device=dev),
                        unit=torch.empty(n_trials, dtype=torch.int32, device=dev))
            tr = nd_mc_trace(tr_t["dE"].data_ptr(), tr_t["sabs"].data_ptr(),
                             tr_t["accepted"].data_ptr(), tr_t["unit"].data_ptr())
        st = nd_mc_stats() if stats else None
        p = params.c()
        self.version += 1
        _check(lib().nd_mc_sweep(self.handle, C.byref(p), C.c_uint64(seed), C.c_uint64(first_trial),
                                 int(n_trials), C.byref(st) if st is not None else None,
                                 C.byref(tr) if tr is not None else None))
        out = {}
        if st is not None:
            out.update(trials=st.trials, accepted=st.accepted, near_ties=st.near_ties,
                       E_total=st.E_total, dE_sum=st.dE_sum)
        if tr_t is not None:
            out["trace"] = tr_t
        return out


class Batch:
    """Several boxes run as one HIP graph (nd_batch_*): Metropolis sweeps,
    pair histograms, g(r) and S(Q) of every box in shared launches."""

    def __init__(self, boxes):
        self.boxes = list(boxes)
        n = len(self.boxes)
        for b in self.boxes:
            b._sync_stream()
        arr = (C.c_void_p * n)(*[b.handle.value for b in self.boxes])
        h = C.c_void_p()
        _check(lib().nd_batch_create(arr, n, C.byref(h)))
        self._h = h
        _live_batches.add(self)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().nd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        """(graph captures, graph launches) so far."""
        c = C.c_int64()
        n = C.c_int64()
        _check(lib().nd_batch_info(self._h, C.byref(c), C.byref(n)))
        return c.value, n.value

    def run(self, sweeps, params, seeds, first_trials, dr=None, nbins=None, w=None, self_term=None,
            Q=None, counts=None, g=None, S=None, stats=False, trace=False):
        """One run.  params/seeds/first_trials/nbins/self_term: one per box; w: [n, P];
        counts/g/S: lists of device tensors ([P, nbins_i] int64, [P, nbins_i] float64,
        [nQ] float64), or None to skip that stage.  trace=True records every
        trial of every box (returned under "trace" of each box's stats)."""
        torch = _torch()
        n = len(self.boxes)
        for b in self.boxes:
            b._sync_stream()
        keep = []
        pl = nd_batch_plan()
        pl.sweeps = int(sweeps)
        if sweeps > 0:
            mcs = (nd_mc_params * n)(*[p.c() for p in params])
            sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
            ft = np.ascontiguousarray(np.asarray(first_trials, dtype=np.uint64))
            keep += [mcs, sd, ft]
            pl.mc = C.cast(mcs, C.c_void_p)
            pl.seed = sd.ctypes.data
            pl.first_trial = ft.ctypes.data
        if counts is not None:
            nb = np.ascontiguousarray(np.asarray(nbins, dtype=np.int32))
            cp = (C.c_void_p * n)(*[c.data_ptr() for c in counts])
            keep += [nb, cp]
            pl.dr = float(dr)
            pl.nbins = nb.ctypes.data
            pl.counts = C.cast(cp, C.c_void_p)
            if g is not None:
                gp = (C.c_void_p * n)(*[x.data_ptr() for x in g])
                keep.append(gp)
                pl.g = C.cast(gp, C.c_void_p)
                if S is not None and Q is not None:
                    Qd = Q.to(dtype=torch.float64).contiguous()
                    ww = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
                    st = np.ascontiguousarray(np.asarray(self_term, dtype=np.float64))
                    sp = (C.c_void_p * n)(*[x.data_ptr() for x in S])
                    keep += [Qd, ww, st, sp]
                    pl.Q = Qd.data_ptr()
                    pl.nQ = int(Qd.shape[0])
                    pl.w = ww.ctypes.data
                    pl.self_term = st.ctypes.data
                    pl.S = C.cast(sp, C.c_void_p)
        tr_t = None
        if trace and sweeps > 0:
            tr_t, trs = [], []
            for b in self.boxes:
                nt = int(sweeps) * b.n_units
                dev = f"cuda:{b.device}"
                d = dict(dE=torch.empty(nt, dtype=torch.float64, device=dev),
                         sabs=torch.empty(nt, dtype=torch.float64, device=dev),
                         accepted=torch.empty(nt, dtype=torch.uint8, device=dev),
                         unit=torch.empty(nt, dtype=torch.int32, device=dev))
                tr_t.append(d)
                trs.append(nd_mc_trace(d["dE"].data_ptr(), d["sabs"].data_ptr(), d["accepted"].data_ptr(),
                                       d["unit"].data_ptr()))
            tra = (nd_mc_trace * n)(*trs)
            keep.append(tra)
            pl.trace = C.cast(tra, C.c_void_p)
            stats = True
        sts = (nd_mc_stats * n)() if stats else None
        if sweeps > 0:
            for b in self.boxes:
                b.version += 1
        _check(lib().nd_batch_run(self._h, C.byref(pl), C.cast(sts, C.c_void_p) if sts is not None else None))
        if sts is None:
            return None
        out = [dict(trials=x.trials, accepted=x.accepted, near_ties=x.near_ties, E_total=x.E_total,
                    dE_sum=x.dE_sum) for x in sts]
        if tr_t is not None:
            for o, d in zip(out, tr_t):
                o["trace"] = d
        return out


def pair_histogram(box: Box, dr: float, nbins: int, out=None):
    """Exact pair counts [P, nbins] (int64 device tensor holding the uint64 counts)."""
    torch = _torch()
    box._sync_stream()
    if out is None:
        out = torch.empty((box.P, nbins), dtype=torch.int64, device=f"cuda:{box.device}")
    _check(lib().nd_pair_histogram(box.handle, float(dr), int(nbins), _dptr(out), ND_DEVICE))
    return out


def gr_normalize(counts, dr, V, npairs):
    torch = _torch()
    P, nb = counts.shape
    g = torch.empty((P, nb), dtype=torch.float64, device=counts.device)
    npairs = _host_f64(npairs, P)
    if counts.dtype == torch.int64:
        _check(lib().nd_gr_normalize(_dptr(counts.contiguous()), P, nb, float(dr), float(V),
                                     npairs.ctypes.data, _dptr(g), ND_DEVICE, _stream()))
    else:
        raise TypeError("counts must be the int64 tensor returned by pair_histogram")
    return g


def sq_transform(g, dr, rho, w, self_term, Q):
    torch = _torch()
    g = g.contiguous()
    P, nb = g.shape
    Q = Q.to(device=g.device, dtype=torch.float64).contiguous()
    S = torch.empty(Q.shape[0], dtype=torch.float64, device=g.device)
    w = _host_f64(w, P)
    _check(lib().nd_sq_transform(_dptr(g), P, nb, float(dr), float(rho), w.ctypes.data,
                                 float(self_term), _dptr(Q), Q.shape[0], _dptr(S), ND_DEVICE,
                                 _stream()))
    return S


def sq_adjoint(dLdS, nbins, dr, rho, V, w, npairs, Q):
    torch = _torch()
    dLdS = dLdS.to(torch.float64).contiguous()
    Q = Q.to(device=dLdS.device, dtype=torch.float64).contiguous()
    w = _host_f64(w)
    npairs = _host_f64(npairs, w.shape[0])
    P = w.shape[0]
    A = torch.empty((P, nbins), dtype=torch.float64, device=dLdS.device)
    _check(lib().nd_sq_adjoint(_dptr(dLdS), P, int(nbins), float(dr), float(rho), float(V),
                               w.ctypes.data, npairs.ctypes.data, _dptr(Q), Q.shape[0], _dptr(A),
                               ND_DEVICE, _stream()))
    return A


def hist_broad(box: Box, dr, nbins, sigma):
    torch = _torch()
    box._sync_stream()
    out = torch.empty((box.P, nbins), dtype=torch.float64, device=f"cuda:{box.device}")
    _check(lib().nd_hist_broad(box.handle, float(dr), int(nbins), float(sigma), _dptr(out), ND_DEVICE))
    return out


def hist_broad_backward(box: Box, dr, nbins, sigma, A):
    torch = _torch()
    box._sync_stream()
    A = A.to(torch.float64).contiguous()
    out = torch.empty((3, box.N), dtype=torch.float64, device=f"cuda:{box.device}")
    _check(lib().nd_hist_broad_backward(box.handle, float(dr), int(nbins), float(sigma), _dptr(A),
                                        _dptr(out), ND_DEVICE))
    return out


def forces(box: Box):
    """(dE/dx [3, N] float64 device tensor, E)."""
    torch = _torch()
    box._sync_stream()
    out = torch.empty((3, box.N), dtype=torch.float64, device=f"cuda:{box.device}")
    E = C.c_double()
    _check(lib().nd_forces(box.handle, _dptr(out), C.byref(E), ND_DEVICE))
    return out, E.value


def forces_noalloc(box: Box, dEdx, E=None):
    """nd_forces_noalloc into caller tensors: dEdx float64 [3, N] and E float64
    [1] (or None) on the box's device; the library allocates nothing."""
    torch = _torch()
    box._sync_stream()
    if dEdx.dtype != torch.float64 or tuple(dEdx.shape) != (3, box.N) or not dEdx.is_contiguous():
        raise ValueError("dEdx must be a contiguous float64 [3, N] device tensor")
    if E is not None and (E.dtype != torch.float64 or E.numel() < 1):
        raise ValueError("E must be a float64 device tensor of at least one element")
    _check(lib().nd_forces_noalloc(box.handle, _dptr(dEdx), _dptr(E) if E is not None else None))


@dataclass
class EmpParams:
    """Parameters of one empirical-potential update (nd_emp_params)."""
    kT: float
    sigma: float = 0.3
    n_terms: int = 30
    feedback: float = 1.0
    ridge: float = 1e-6
    id_weight: float = 1.0
    emp_max: float = 0.0

    def c(self):
        return nd_emp_params(self.sigma, self.n_terms, 0, self.feedback, self.kT, self.ridge, self.id_weight,
                             self.emp_max)


def emp_update(box: Box, params: EmpParams, W, self_terms, g, dr, Q, S_exp):
    """One EMP update of the box's tables from measured profiles S_exp [n_prof, nQ]
    (device tensor), their Eq. 1 weights W [n_prof, P] and flat terms, and the
    model's g [P, nbins].  Returns (dS [n_prof, nQ], EMP [P, n_pts],
    coefficients [P, n_terms]) as device tensors."""
    torch = _torch()
    box._sync_stream()
    W = np.ascontiguousarray(np.asarray(W, dtype=np.float64))
    st = _host_f64(self_terms, W.shape[0])
    g = g.to(torch.float64).contiguous()
    Q = Q.to(device=g.device, dtype=torch.float64).contiguous()
    S_exp = S_exp.to(device=g.device, dtype=torch.float64).contiguous()
    n_prof, nQ = S_exp.shape
    dS = torch.empty((n_prof, nQ), dtype=torch.float64, device=g.device)
    emp = torch.empty((box.P, box._n_pts), dtype=torch.float64, device=g.device)
    coef = torch.empty((box.P, params.n_terms), dtype=torch.float64, device=g.device)
    p = params.c()
    box.version += 1
    _check(lib().nd_emp_update(box.handle, C.byref(p), n_prof, W.ctypes.data, st.ctypes.data, _dptr(g),
                               g.shape[1], float(dr), _dptr(Q), nQ, _dptr(S_exp), _dptr(dS), _dptr(emp),
                               _dptr(coef)))
    return dS, emp, coef


def refine(box: Box, mc: MCParams, seed: int, W, self_terms, S_exp, Q, dr, nbins, emp: EmpParams,
           iterations: int, sweeps: int, sample_sweeps: int, first_trial: int = 0):
    """The empirical-potential Monte Carlo loop (Sec. "NeuDATool Algorithmic
    Flow", steps MC, "Calculate g(r), S(Q) and EMP" and EPMC): each iteration
    runs `sweeps` sweeps of which the last `sample_sweeps` are accumulated into
    the mean histogram (the running Delta N(r) histogram), turns it into g(r),
    and updates the EMP from the measured profiles S_exp [n_prof, nQ] with
    Eq. 1 weights W [n_prof, P] and flat terms.  Every step runs in the
    library; this function only sequences the calls.  Returns per iteration
    the chi^2 of each profile before its update, and the next trial counter."""
    torch = _torch()
    V, rho = box.density()
    npairs = pair_counts_total(box)
    Qd = torch.as_tensor(Q, device=f"cuda:{box.device}", dtype=torch.float64)
    Sx = torch.as_tensor(S_exp, device=Qd.device, dtype=torch.float64)
    W = np.ascontiguousarray(np.asarray(W, dtype=np.float64))
    history = []
    t = first_trial
    for _ in range(iterations):
        box.track_histogram(dr, nbins)  # restarts the sums
        for s in range(sweeps):
            box.mc_sweep(mc, seed, t, box.n_units, stats=False)
            t += box.n_units
            if s >= sweeps - sample_sweeps:
                box.accumulate()
        mean, _ = box.accumulated()
        g = gr_normalize_f64(mean, dr, V, npairs)
        chi = []
        for i in range(W.shape[0]):
            S = sq_transform(g, dr, rho, W[i], float(self_terms[i]), Qd)
            c2, _ = chi2(S, Sx[i])
            chi.append(float(c2[0]))
        history.append(chi)
        emp_update(box, emp, W, self_terms, g, dr, Qd, Sx)
    box.track_histogram(dr, 0)
    return history, t


def pair_counts_total(box: Box):
    """Number of distinct pairs per pair type (nd_box_pair_counts)."""
    out = np.zeros(box.P)
    _check(lib().nd_box_pair_counts(box.handle, out.ctypes.data))
    return out


def eq1_weights(box: Box, b):
    """Eq. 1 partial weights and flat term for scattering lengths b (nd_eq1_weights)."""
    bb = _host_f64(b, box.M)
    w = np.zeros(box.P)
    flat = C.c_double()
    _check(lib().nd_eq1_weights(box.handle, bb.ctypes.data, w.ctypes.data, C.byref(flat)))
    return w, flat.value


def chi2(S, S_target):
    """(chi^2 = sum (S - S_t)^2 as a 1-element device tensor, dchi^2/dS)."""
    torch = _torch()
    S = S.to(torch.float64).contiguous()
    St = S_target.to(device=S.device, dtype=torch.float64).contiguous()
    out = torch.empty(1, dtype=torch.float64, device=S.device)
    grad = torch.empty_like(S)
    _check(lib().nd_chi2(_dptr(S), _dptr(St), S.shape[0], _dptr(out), _dptr(grad), ND_DEVICE, _stream()))
    return out, grad


def gr_normalize_f64(counts, dr, V, npairs):
    torch = _torch()
    counts = counts.to(torch.float64).contiguous()
    P, nb = counts.shape
    g = torch.empty_like(counts)
    npairs = _host_f64(npairs, P)
    _check(lib().nd_gr_normalize_f64(_dptr(counts), P, nb, float(dr), float(V), npairs.ctypes.data,
                                     _dptr(g), ND_DEVICE, _stream()))
    return g


def _make_autograd():
    import torch

    class Chi2Fn(torch.autograd.Function):
        """chi^2 of the Gaussian-broadened S(Q) against a target, differentiable in xyz.

        Forward: nd_hist_broad -> nd_gr_normalize_f64 -> nd_sq_transform -> nd_chi2.
        Backward: dchi^2/dS -> nd_sq_adjoint -> nd_hist_broad_backward.
        """

        @staticmethod
        def forward(ctx, xyz, box, dr, nbins, sigma, Q, S_target, b):
            # new coordinates: the box's running energy is stale from here
            box.set_coords(xyz, keep_energy=False)
            nh = hist_broad(box, dr, nbins, sigma)
            npairs = pair_counts_total(box)
            V, rho = box.density()
            w, self_term = eq1_weights(box, b)
            g = gr_normalize_f64(nh, dr, V, npairs)
            S = sq_transform(g, dr, rho, w, self_term, Q)
            c2, dS = chi2(S, S_target)
            ctx.save_for_backward(dS, Q, xyz)
            ctx.box, ctx.dr, ctx.nbins, ctx.sigma = box, dr, nbins, sigma
            ctx.rho, ctx.V, ctx.w, ctx.npairs = rho, V, w, npairs
            ctx.version = box.version
            return c2[0]

        @staticmethod
        def backward(ctx, grad_out):
            dS, Q, xyz = ctx.saved_tensors
            # the gradient is taken at the x forward saw: restore it if the
            # box has moved on since (another forward, a sweep, set_coords)
            if ctx.box.version != ctx.version:
                ctx.box.set_coords(xyz, keep_energy=False)
            A = sq_adjoint(dS, ctx.nbins, ctx.dr, ctx.rho, ctx.V, ctx.w, ctx.npairs, Q)
            gx = hist_broad_backward(ctx.box, ctx.dr, ctx.nbins, ctx.sigma, A)
            return (grad_out * gx).to(xyz.dtype), None, None, None, None, None, None, None

    class EnergyFn(torch.autograd.Function):
        """Total energy of the box at xyz; backward gives dE/dx from nd_forces."""

        @staticmethod
        def forward(ctx, xyz, box):
            box.set_coords(xyz, keep_energy=False)
            grad, E = forces(box)
            ctx.save_for_backward(grad)
            ctx.x_dtype = xyz.dtype
            return torch.tensor(E, dtype=torch.float64, device=xyz.device)

        @staticmethod
        def backward(ctx, grad_out):
            (grad,) = ctx.saved_tensors
            return (grad_out * grad).to(ctx.x_dtype), None

    return Chi2Fn, EnergyFn


class _Lazy:
    def __init__(self, idx):
        self.idx = idx
        self._cls = None

    def _get(self):
        if self._cls is None:
            self._cls = _make_autograd()[self.idx]
        return self._cls

    def apply(self, *args):
        return self._get().apply(*args)


Chi2Fn = _Lazy(0)
EnergyFn = _Lazy(1)
