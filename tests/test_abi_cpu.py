"""The C ABI library loads on a host without a GPU, exports every function
include/neuda.h declares, and rejects bad arguments before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "neuda.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:nd_status|int32_t|const char \*)\s*(nd_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    import paper_1904_08756_amd as nd
    if not os.path.exists(nd.LIB_PATH):
        pytest.fail("libneuda.so is not built (run __graft_entry__.build())")
    return nd.lib()


def test_header_declares_the_api():
    fns = declared_functions()
    for name in ("nd_box_create", "nd_mc_sweep", "nd_pair_histogram", "nd_sq_transform",
                 "nd_hist_broad", "nd_hist_broad_backward", "nd_forces", "nd_last_error"):
        assert name in fns


def test_every_declared_symbol_is_exported(L):
    import paper_1904_08756_amd as nd
    for name in declared_functions():
        assert hasattr(L, name), name
        assert name in nd.EXPORTS, f"binding lacks {name}"


def test_abi_version(L):
    assert L.nd_abi_version() == 1


def _desc(nd, xyz, sp, offs, L_, M):
    return nd.nd_box_desc(xyz.shape[1], M, L_, sp.ctypes.data, offs.shape[0] - 1, offs.ctypes.data,
                          xyz.ctypes.data, 0, None)


@pytest.mark.parametrize("case", ["null", "n1", "species", "outside", "nan", "offsets", "bigunit", "L"])
def test_box_create_validation(L, case):
    import paper_1904_08756_amd as nd
    xyz = np.array([[1.0, 2.0, 3.0], [1.0, 1.0, 1.0], [1.0, 1.0, 1.0]], np.float32)
    sp = np.array([0, 1, 0], np.uint8)
    offs = np.array([0, 1, 3], np.int32)
    Lb, M = 10.0, 2
    if case == "n1":
        xyz = xyz[:, :1].copy(); sp = sp[:1].copy(); offs = np.array([0, 1], np.int32)
    elif case == "species":
        sp = np.array([0, 2, 0], np.uint8)
    elif case == "outside":
        xyz[0, 2] = 10.0
    elif case == "nan":
        xyz[1, 1] = np.nan
    elif case == "offsets":
        offs = np.array([0, 2, 2, 3], np.int32)
    elif case == "bigunit":
        xyz = np.ones((3, 9), np.float32); sp = np.zeros(9, np.uint8); offs = np.array([0, 9], np.int32)
    elif case == "L":
        Lb = -1.0
    h = C.c_void_p()
    if case == "null":
        rc = L.nd_box_create(None, C.byref(h))
    else:
        d = _desc(nd, np.ascontiguousarray(xyz), sp, offs, Lb, M)
        rc = L.nd_box_create(C.byref(d), C.byref(h))
    assert rc == -1
    assert h.value is None
    assert len(L.nd_last_error()) > 0


def test_stateless_entry_points_validate(L):
    g = np.zeros(30)
    S = np.zeros(5)
    Q = np.ones(5)
    w = np.ones(3)
    npairs = np.ones(3)
    # P out of range, nbins 0, negative dr, bad where, NULL pointers
    assert L.nd_sq_transform(g.ctypes.data, 0, 10, 0.1, 0.1, w.ctypes.data, 0.0, Q.ctypes.data, 5,
                             S.ctypes.data, 0, None) == -1
    assert L.nd_sq_transform(g.ctypes.data, 3, 0, 0.1, 0.1, w.ctypes.data, 0.0, Q.ctypes.data, 5,
                             S.ctypes.data, 0, None) == -1
    assert L.nd_sq_transform(g.ctypes.data, 3, 10, -0.1, 0.1, w.ctypes.data, 0.0, Q.ctypes.data, 5,
                             S.ctypes.data, 0, None) == -1
    assert L.nd_sq_transform(g.ctypes.data, 3, 10, 0.1, 0.1, w.ctypes.data, 0.0, Q.ctypes.data, 5,
                             S.ctypes.data, 7, None) == -1
    assert L.nd_gr_normalize(None, 3, 10, 0.1, 1.0, npairs.ctypes.data, g.ctypes.data, 0, None) == -1
    npairs[1] = 0.0
    c = np.zeros(30, np.uint64)
    assert L.nd_gr_normalize(c.ctypes.data, 3, 10, 0.1, 1.0, npairs.ctypes.data, g.ctypes.data, 0, None) == -1
    assert L.nd_chi2(None, None, 5, None, None, 0, None) == -1
    assert L.nd_pair_histogram(None, 0.1, 10, c.ctypes.data, 0) == -1
    assert L.nd_mc_sweep(None, None, 0, 0, 1, None, None) == -1
    assert L.nd_box_destroy(None) == 0
    h = C.c_void_p()
    assert L.nd_batch_create(None, 0, C.byref(h)) == -1 and h.value is None
    assert L.nd_batch_create(None, 3, C.byref(h)) == -1
    assert L.nd_batch_run(None, None, None) == -1
    assert L.nd_batch_info(None, None, None) == -1
    assert L.nd_batch_destroy(None) == 0
    n = C.c_size_t(0)
    assert L.nd_box_save(None, None, C.byref(n)) == -1
    assert L.nd_box_load(None, None, 0) == -1


def test_product_path_does_not_import_oracle():
    import subprocess
    import sys
    code = ("import sys, paper_1904_08756_amd as nd; nd.lib(); "
            "assert 'oracle' not in sys.modules, 'binding imported the oracle'")
    subprocess.check_call([sys.executable, "-c", code], cwd=ROOT)
    for dirpath, _, files in os.walk(os.path.join(ROOT, "paper_1904_08756_amd")):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "orc_" not in text, f
