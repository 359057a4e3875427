"""Checkpoint and resume of the Metropolis state (nd_box_save/nd_box_load).

A box restored from a checkpoint taken after t trials and run on from
trial t repeats, bit for bit, the original box run on from the same point
(coordinates, running energy, acceptance count): the image carries the
coordinates, the running energy and the cell lists with their drift
bookkeeping.  Against one uninterrupted call over all trials the batch
boundaries differ, so the energy sums may differ in rounding only; the
coordinates agree exactly because every decision is the same.
"""
import numpy as np
import pytest

import synthetic as syn

pytestmark = pytest.mark.gpu


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


def _box(nd, sbox, T):
    g = nd.Box.from_synthetic(sbox)
    g.set_tables(T.U, T.h, T.r_cut)
    g.total_energy()
    return g


@pytest.mark.parametrize("cfg,n1,n2", [("c1", 777, 1500), ("c4small", 1234, 3000)])
def test_resume_is_bit_exact(nd, cfg, n1, n2):
    if cfg == "c1":
        sbox, T, mc = syn.config_c1()
    else:
        boxes, T, mc = syn.config_c4()
        sbox = min(boxes, key=lambda b: b.n_atoms)
    say("checkpoint", cfg, sbox.n_atoms, n1, n2)
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])
    seed = 4242
    a = _box(nd, sbox, T)
    a.mc_sweep(p, seed, 0, n1)
    img = a.save()
    ra = a.mc_sweep(p, seed, n1, n2)
    b = _box(nd, sbox, T)
    b.load(img)
    rb = b.mc_sweep(p, seed, n1, n2)
    assert np.array_equal(a.coords_host(), b.coords_host())
    assert ra["E_total"] == rb["E_total"]
    assert ra["accepted"] == rb["accepted"] and ra["dE_sum"] == rb["dE_sum"]
    # one uninterrupted call over the same trials
    c = _box(nd, sbox, T)
    rc = c.mc_sweep(p, seed, 0, n1 + n2)
    assert np.array_equal(c.coords_host(), b.coords_host())
    assert abs(rc["E_total"] - rb["E_total"]) <= 1e-9 * max(1.0, abs(rc["E_total"]))


def test_checkpoint_without_cells_and_rejections(nd):
    sbox, T, mc = syn.config_c1()
    a = _box(nd, sbox, T)
    img = a.save()  # no Metropolis call yet: no cell lists in the image
    b = _box(nd, sbox, T)
    b.set_coords(np.zeros((3, sbox.n_atoms), np.float32))
    b.load(img)
    assert np.array_equal(a.coords_host(), b.coords_host())
    assert b.energy() == a.energy()
    p = nd.MCParams(mc["kT"], mc["max_disp"], mc["max_rot"])
    a.mc_sweep(p, 1, 0, 500)
    img = bytearray(a.save())
    bad = bytearray(img)
    bad[len(bad) // 2] ^= 0x10
    with pytest.raises(nd.NeudaError, match="hash"):
        b.load(bytes(bad))
    with pytest.raises(nd.NeudaError, match="truncated"):
        b.load(bytes(img[:-9]))
    other = syn.water_box(301, 20.8, 5, "other")
    c = nd.Box.from_synthetic(other)
    with pytest.raises(nd.NeudaError, match="different box"):
        c.load(bytes(img))
    b.load(bytes(img))
    assert np.array_equal(a.coords_host(), b.coords_host())
