"""Simulations at the size limit.  In 2D a simulation's whole population
block (three lattices in runs of 64 nodes) must fit one 32-bit buffer range:
the largest FP32 coupled drop tested holds 2.12 GB.  In 3D a lattice must fit
one 32-bit range, and the flow lattice g starts 2 lattices into a
simulation's block, beyond a 32-bit byte offset.

One step of a coupled shear drop at that size is checked window by window
against the FP64 oracle: a node's next pre-collision populations depend on
the current ones within radius 3 (pull 1, normals 1, phi stencil 1), so the
oracle, run one step on a periodic 44 x 44 (x 44) window cut from the GPU's
populations, must reproduce the GPU's result on the window's interior
(margin 6; exact in FP64 on the CPU from radius 3 on).  One window sits on
the drop's interface, one in the sheared bulk (where f is zero: differences
are scaled by max(|populations|, 1e-2))."""
import gc

import numpy as np
import pytest

from paper_2504_09024_amd import workloads as W

pytestmark = pytest.mark.gpu

WIN, MARGIN = 44, 6


def _window2(a, x0, y0):
    return np.ascontiguousarray(a[:, y0:y0 + WIN, x0:x0 + WIN])


def _window3(a, x0, y0, z0):
    return np.ascontiguousarray(a[:, z0:z0 + WIN, y0:y0 + WIN, x0:x0 + WIN])


def test_2d_simulation_at_the_2gib_limit_fp32(oracle_mod, gpu_lib):
    """4096 x 4800 coupled shear drop in FP32: a 2.12 GB population block,
    within 1.2% of the 2^31-byte limit (one more row of 4096 nodes fits, the
    next size up is rejected)."""
    from paper_2504_09024_amd import cmlb
    nx, ny = 4096, 4800
    assert 27 * nx * ny * 4 < 2 ** 31 <= 27 * nx * (ny + 64) * 4
    p, fl = W.shear_drop(nx=nx, ny=ny, R=64.0, Re=1.0)
    ctx = cmlb.Context(p, "fp32")
    ctx.init_fields(0, fl["phi"], fl["c"], fl["ux"], fl["uy"])
    del fl
    gc.collect()
    # windows: right edge of the drop; a wall-free interior strip of the shear
    wins = [(nx // 2 + 64 - WIN // 2, ny // 2 - WIN // 2), (1000, 3000)]
    pre = [[_window2(a, x0, y0) for a in ctx.get_populations(0)] for x0, y0 in wins]
    gc.collect()
    ctx.step(1)
    post = [[_window2(a, x0, y0) for a in ctx.get_populations(0)] for x0, y0 in wins]
    assert ctx.fault_flags(0) == 0
    ctx.close()
    gc.collect()
    wp = dict(p, nx=WIN, ny=WIN, bc_y="periodic")
    for (f, h, g), (gf, gh, gg) in zip(pre, post):
        o = oracle_mod.OracleSim.from_populations(oracle_mod.make_params(**wp), f, h, g)
        assert o.run(1) == 0
        for a, b in ((gf, o.f), (gh, o.h), (gg, o.g)):
            sl = (slice(None), slice(MARGIN, WIN - MARGIN), slice(MARGIN, WIN - MARGIN))
            d = np.abs(a[sl] - b[sl]).max() / max(np.abs(b[sl]).max(), 1e-2)
            print(f"2D window one-step max rel diff {d:.2e}", flush=True)
            assert d <= 1e-6, d


def test_3d_lattice_above_1gib_fp32(oracle_mod, gpu_lib):
    """256 x 256 x 160 coupled drop in shear in FP32: 1.13 GB per lattice."""
    from paper_2504_09024_amd import cmlb
    nx, ny, nz = 256, 256, 160
    assert 27 * nx * ny * nz * 4 > 2 ** 30
    p, fl = W.shear_drop3(nx=nx, ny=ny, nz=nz, R=32.0, Re=1.0)
    ctx = cmlb.Context3(p, "fp32")
    ctx.init_fields(0, fl["phi"], fl["c"], fl["ux"], fl["uy"], fl["uz"])
    del fl
    gc.collect()
    wins = [(nx // 2 + 32 - WIN // 2, ny // 2 - WIN // 2, nz // 2 - WIN // 2), (10, 100, 100)]
    pre = [[_window3(a, *w) for a in ctx.get_populations(0)] for w in wins]
    gc.collect()
    ctx.step(1)
    post = [[_window3(a, *w) for a in ctx.get_populations(0)] for w in wins]
    assert ctx.fault_flags(0) == 0
    ctx.close()
    gc.collect()
    wp = dict(p, nx=WIN, ny=WIN, nz=WIN, bc_y="periodic")
    for (f, h, g), (gf, gh, gg) in zip(pre, post):
        o = oracle_mod.OracleSim3.from_populations(oracle_mod.make_params3(**wp), f, h, g)
        assert o.run(1) == 0
        m = slice(MARGIN, WIN - MARGIN)
        for a, b in ((gf, o.f), (gh, o.h), (gg, o.g)):
            sl = (slice(None), m, m, m)
            d = np.abs(a[sl] - b[sl]).max() / max(np.abs(b[sl]).max(), 1e-2)
            print(f"3D window one-step max rel diff {d:.2e}", flush=True)
            assert d <= 1e-6, d
