"""cmlb_inventories_noalloc, the allocation-free form of cmlb_inventories
(scratch in the library's static device array), called through the C ABI:
its totals are bitwise those of cmlb_inventories on two calls in a row, the
second over a smaller range (fewer rows) than the first, and sizes beyond
the scratch array are rejected."""
import numpy as np
import pytest

from paper_2504_09024_amd import workloads as W
from parity_util import gpu_ctx

pytestmark = pytest.mark.gpu


def _device_sums(ctx, torch, first, n, stream_sync=True):
    d = torch.full((2 * n,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ctx.inventories_noalloc(d.data_ptr(), first, n)
    ctx.synchronize()
    return d.cpu().numpy().reshape(n, 2)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_noalloc_inventories_match_allocating_entry_point(gpu_lib, prec):
    import torch
    sims = [W.shear_drop(nx=nx, ny=ny, R=ny / 8, Ca=ca, E=e, c0=c0)
            for nx, ny, ca, e, c0 in ((256, 160, 0.2, 0.1, 0.2), (200, 96, 0.5, 0.4, 0.4),
                                      (64, 48, 0.1, 0.3, 0.1), (100, 70, 0.3, 0.2, 0.3))]
    ctx = gpu_ctx([s[0] for s in sims], [s[1] for s in sims], prec)
    ctx.step(9)
    ref_all = ctx.inventories()
    # first call: every simulation (374 rows); second: a smaller range that
    # leaves stale partials of the first call in the rest of the array
    got_all = _device_sums(ctx, torch, 0, 4)
    got_two = _device_sums(ctx, torch, 2, 2)
    print(prec, got_all.tolist())
    assert np.array_equal(got_all, ref_all)
    assert np.array_equal(got_two, ctx.inventories(2, 2))
    assert np.array_equal(got_two, ref_all[2:4])
    # after more steps the same calls follow the new state
    ctx.step(5)
    assert np.array_equal(_device_sums(ctx, torch, 1, 1), ctx.inventories(1, 1))
    ctx.close()


def test_noalloc_inventories_reject_oversized_and_bad_arguments(gpu_lib):
    import torch
    from paper_2504_09024_amd import cmlb
    # 65537 rows: one more than the scratch array holds
    p, fl = W.static_drop(n=64, R=16.0)
    ps = [dict(p, ny=65537 // 7 + (1 if i < 65537 % 7 else 0)) for i in range(7)]
    assert sum(q["ny"] for q in ps) == 65537
    ctx = cmlb.Context(ps, "fp32")
    d = torch.zeros(2 * 7, dtype=torch.float64, device="cuda")
    with pytest.raises(cmlb.CmlbError) as e:
        ctx.inventories_noalloc(d.data_ptr(), 0, 7)
    assert "scratch" in str(e.value)
    with pytest.raises(cmlb.CmlbError):
        ctx.inventories_noalloc(0, 0, 1)
    with pytest.raises(cmlb.CmlbError):
        ctx.inventories_noalloc(d.data_ptr() + 4, 0, 1)
    with pytest.raises(cmlb.CmlbError):
        ctx.inventories_noalloc(d.data_ptr(), 5, 3)
    ctx.close()
