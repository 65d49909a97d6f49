"""The allocation-free moments entry point (dvm_get_moments_noalloc) against
dvm_get_moments on the same converged states: two calls in a row, the
second on a smaller instance, outputs in caller-owned device tensors, and no
allocation through the context's allocator hooks during the calls."""
import numpy as np
import pytest

from paper_1704_03126_amd.geometry import porous_discs, rough_channel

pytestmark = pytest.mark.gpu

MOMENTS = ("rho", "u1", "u2", "tau", "p12")


@pytest.fixture(scope="module")
def dvm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1704_03126_amd.dvm as d
    d.load_library()
    return d


def test_noalloc_moments_match_the_allocating_entry_point(dvm):
    import torch
    big = porous_discs(96, 0.6, 91)               # 2 strips, periodic
    small = rough_channel(40, 24, 5, 20)           # 1 strip, walls, Maxwell below
    nv = 12
    alloc = dvm.TorchAllocator()
    s = dvm.Solver(nv, 2, tol=1e-11, allocator=alloc)
    s.set_geometry(0, big.mask, big.periodic_y, big.cells_per_H)
    s.set_geometry(1, small.mask, small.periodic_y, small.cells_per_H)
    s.solve(0, 1.3)
    s.solve(1, 0.7, 0.85)
    torch.cuda.synchronize()
    for inst, g in ((0, big), (1, small)):        # second call: the smaller input
        ref = s.moments(inst, shear=True)
        out = {m: torch.full((g.ny, g.nx), float("nan"), dtype=torch.float64, device="cuda")
               for m in MOMENTS}
        calls = alloc.calls
        s.moments_into(inst, **out)
        torch.cuda.synchronize()
        assert alloc.calls == calls                # nothing allocated by the call
        for m in MOMENTS:
            got = out[m].cpu().numpy()
            assert np.all(np.isfinite(got)), m
            assert np.max(np.abs(got - ref[m])) <= 1e-14 * max(1.0, np.max(np.abs(ref[m]))), m
        assert np.max(np.abs(ref["tau"])) > 1e-4 and np.max(np.abs(ref["p12"])) > 1e-4
    # a subset of outputs, after the two calls above: the others stay as they were
    u1 = torch.zeros((small.ny, small.nx), dtype=torch.float64, device="cuda")
    s.moments_into(1, u1=u1)
    torch.cuda.synchronize()
    assert np.array_equal(u1.cpu().numpy(), s.moments(1)["u1"])
    with pytest.raises(ValueError):
        s.moments_into(1, u1=torch.zeros((3, 3), dtype=torch.float64, device="cuda"))
    s.close()
    assert alloc.bytes_held == 0
