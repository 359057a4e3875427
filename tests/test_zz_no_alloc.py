"""nd_forces_noalloc, the allocation-free variant of nd_forces, through the
C ABI: on two calls in a row (the second on a smaller box, so the shared
scratch holds the first call's sums beforehand) it gives nd_forces's
gradient and energy bit for bit (both sum the pair terms as integers), and
within the forces' oracle tolerance of the FP64 oracle; boxes beyond the
scratch's atom limit are refused."""
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


def _check_box(nd, orc, box, T):
    import torch
    g = nd.Box.from_synthetic(box)
    g.set_tables(T.U, T.h, T.r_cut)
    want, E_want = nd.forces(g)
    got = torch.full((3, box.n_atoms), float("nan"), dtype=torch.float64, device="cuda")
    E = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    nd.forces_noalloc(g, got, E)
    torch.cuda.synchronize()
    assert torch.equal(got, want), "gradient differs from nd_forces"
    assert float(E[0]) == E_want, "energy differs from nd_forces"
    ref, E_o = orc.forces(box, T)
    scale = np.abs(ref).max()
    assert np.all(np.abs(got.cpu().numpy() - ref) <= 1e-9 * scale + 1e-9 * np.abs(ref))
    # E may be omitted
    got2 = torch.empty_like(got)
    nd.forces_noalloc(g, got2)
    torch.cuda.synchronize()
    assert torch.equal(got2, want)
    g.close()


def test_noalloc_forces_equal_nd_forces_two_calls(nd, orc):
    big = syn.water_box(1500, 24.0, 31, "noalloc big")
    small = syn.water_box(400, 16.0, 32, "noalloc small")
    T = syn.water_tables(r_cut=8.0)
    print("noalloc forces: 4500 atoms, then 1200 atoms", flush=True)
    _check_box(nd, orc, big, T)
    _check_box(nd, orc, small, T)


def test_noalloc_forces_refuses_boxes_past_the_limit(nd):
    import torch
    n = 262144 + 1
    box = syn.atomic_box((n,), 140.0, 5, ("X",), "past the limit")
    T = syn.potential_table(1, 8.0, 0.01, [(3.0, 0.5)], [0.0])
    g = nd.Box.from_synthetic(box)
    g.set_tables(T.U, T.h, T.r_cut)
    out = torch.empty((3, n), dtype=torch.float64, device="cuda")
    with pytest.raises(nd.NeudaError, match="RANGE"):
        nd.forces_noalloc(g, out)
    g.close()
