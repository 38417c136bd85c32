"""GPU parity of the 3D (D3Q27) path against the FP64 3D oracle, through
the C ABI of include/cmlb3.h.

Tolerances (relative L2 per field at the final step): FP64 <= 1e-12,
FP32 <= 1e-5 on phi, c, u, FP16 storage <= 1e-3.  Sizes span several
collision columns (64 x 4 or 64 x 8 nodes, one to three z segments) and
64 x 4-row moment tiles with ragged tails in x, y and z, down to a 4 x 4 x 1
grid; the FP64 cases are checked to be well conditioned on the CPU.
"""
import math

import numpy as np
import pytest

from paper_2504_09024_amd import workloads as W
from parity_cases3 import CASES3

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp16": 1e-3}
CS2 = 1.0 / 3.0


def ctx3(p, fl, prec, graph=True):
    from paper_2504_09024_amd import cmlb
    ps, fls = (p, fl) if isinstance(p, list) else ([p], [fl])
    c = cmlb.Context3(ps, prec)
    c.set_use_graph(graph)
    for i, f in enumerate(fls):
        c.init_fields(i, f["phi"], f["c"], f.get("ux"), f.get("uy"), f.get("uz"), f.get("P"))
    return c


def oracle3(oracle_mod, p, fl):
    return oracle_mod.OracleSim3(oracle_mod.make_params3(**p), fl["phi"], fl["c"], fl.get("ux"),
                                 fl.get("uy"), fl.get("uz"), fl.get("P"))


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def errors3(g, o, flow):
    err = {"phi": rel(g["phi"], o["phi"]), "c": rel(g["c"], o["c"])}
    if flow != "none":
        u = lambda r: np.stack([r["ux"], r["uy"], r["uz"]])
        err["u"] = rel(u(g), u(o))
    if flow == "coupled":
        err["P"] = rel(g["P"], o["P"])
    return err


@pytest.mark.parametrize("name", ["static3", "prescribed3", "coupled3"])
def test_init_populations3(oracle_mod, gpu_lib, name):
    build, _ = CASES3[name]
    p, fl = build()
    o = oracle3(oracle_mod, p, fl)
    c = ctx3(p, fl, "fp64")
    f, h, g = c.get_populations(0)
    for a, b in ((f, o.f), (h, o.h)) + (((g, o.g),) if o.g is not None else ()):
        assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()
    c.close()


PARITY3 = [("static3", "fp64"), ("static3", "fp32"), ("prescribed3", "fp64"),
           ("prescribed3", "fp32"), ("coupled3", "fp64"), ("coupled3", "fp32"),
           ("density3", "fp64"), ("shear3", "fp64"), ("shear3", "fp32"),
           ("static3", "fp16"), ("shear3", "fp16"), ("thin3", "fp64"), ("thin3", "fp32"),
           ("tiny3", "fp64"), ("tiny3", "fp32"), ("density3", "fp32"), ("density3", "fp16")]


@pytest.mark.parametrize("name,prec", PARITY3)
def test_parity3(oracle_mod, gpu_lib, name, prec):
    build, steps = CASES3[name]
    p, fl = build()
    o = oracle3(oracle_mod, p, fl)
    c = ctx3(p, fl, prec)
    c.step(steps)
    g = c.read_fields(0)
    assert o.run(steps) == 0
    err = errors3(g, o.fields(), p["flow"])
    print(name, prec, {k: f"{v:.2e}" for k, v in err.items()})
    for k in ("phi", "c", "u"):
        if k in err:
            assert err[k] <= TOL[prec], (k, err[k])
    if prec == "fp64" and "P" in err:
        assert err["P"] <= TOL[prec]
    c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_tile_shapes_bitwise3(gpu_lib, prec):
    """Every collision launch shape (column height, planes per column
    segment; here one segment of 12 planes against a full and a ragged one
    of 8, and three of 4) gives the same populations bit for bit."""
    p, fl = CASES3["coupled3"][0]()
    outs = []
    c0 = ctx3(p, fl, prec)
    shapes = c0.launch_options()
    c0.close()
    assert (4, 16) in shapes and (4, 8) in shapes and len(shapes) >= 3
    for shape in shapes:
        c = ctx3(p, fl, prec)
        c.set_tile_shape(*shape)
        c.step(20)
        outs.append(c.get_populations(0))
        c.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_autotune3_leaves_the_run_unchanged(gpu_lib, prec):
    """The 3D autotuner's trials leave no trace: 10 steps, autotune, 20 steps
    equals 30 plain steps bit for bit, the step counter is kept, and the
    chosen shape is one of the accepted ones."""
    p, fl = CASES3["coupled3"][0]()
    a = ctx3(p, fl, prec)
    a.step(10)
    ty, zs, pol = a.autotune(5)
    assert (ty, zs) in a.launch_options() and pol in ("default", "nt")
    assert a.step_count == 10
    a.step(20)
    b = ctx3(p, fl, prec)
    b.step(30)
    for x, y in zip(a.get_populations(0), b.get_populations(0)):
        assert np.array_equal(x, y)
    assert a.fault_flags(0) == 0
    a.close()
    b.close()


def test_store_policies_bitwise3(gpu_lib):
    """Default and non-temporal population stores give identical results."""
    p, fl = CASES3["coupled3"][0]()
    outs = []
    for pol in ("default", "nt"):
        c = ctx3(p, fl, "fp32")
        c.set_store_policy(pol)
        c.step(10)
        outs.append(c.get_populations(0))
        c.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_zero_steps3(gpu_lib):
    """step(0) launches nothing: populations and the step count unchanged."""
    p, fl = CASES3["coupled3"][0]()
    c = ctx3(p, fl, "fp32")
    c.step(3)
    before = c.get_populations(0)
    c.step(0)
    assert c.step_count == 3
    for a, b in zip(before, c.get_populations(0)):
        assert np.array_equal(a, b)
    c.close()


def test_graph_matches_direct3(gpu_lib):
    p, fl = CASES3["coupled3"][0]()
    outs = []
    for graph in (True, False):
        c = ctx3(p, fl, "fp32", graph=graph)
        for n in (35, 3):
            c.step(n)
        assert c.step_count == 38
        outs.append(c.get_populations(0))
        c.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_batched_matches_single3(gpu_lib):
    cases = [CASES3["coupled3"][0](), W.random_fields3(40, 16, 9, seed=7, amp=1.0, sigma0=1e-3,
                                                       beta=0.2, u_wall=1e-2, M_phi=0.04)]
    c = ctx3([x[0] for x in cases], [x[1] for x in cases], "fp64")
    c.step(30)
    batched = [c.get_populations(i) for i in range(2)]
    c.close()
    for i, (p, fl) in enumerate(cases):
        s = ctx3(p, fl, "fp64")
        s.step(30)
        for a, b in zip(batched[i], s.get_populations(0)):
            assert np.array_equal(a, b)
        s.close()


def test_conservation3_fp64(gpu_lib):
    p, fl = CASES3["coupled3"][0]()
    c = ctx3(p, fl, "fp64")
    s0 = c.inventory(0)
    c.step(400)
    s1 = c.inventory(0)
    assert c.fault_flags(0) == 0
    for a, b in zip(s1, s0):
        assert abs(a - b) / abs(b) < 1e-13, (a, b)
    c.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-6)])
def test_c5_full_size_one_step(oracle_mod, gpu_lib, prec, tol):
    """256 x 128 x 128 coupled shear drop (R = 32, Ca = 0.3, E = 0.2, c0 = 0.3,
    Re = 0.1) in the benchmark's launch configuration: after 20 GPU steps,
    one more step from the GPU's own populations through the oracle."""
    p, fl = W.shear_drop3()
    c = ctx3(p, fl, prec)
    c.step(20)
    f, h, g = c.get_populations(0)
    o = oracle_mod.OracleSim3.from_populations(oracle_mod.make_params3(**p), f, h, g, t=20)
    del f, h, g
    c.step(1)
    assert o.run(1) == 0
    gf, gh, gg = c.get_populations(0)
    for a, b in ((gf, o.f), (gh, o.h), (gg, o.g)):
        d = np.abs(a - b).max() / np.abs(b).max()
        print(prec, f"one-step max rel diff {d:.2e}")
        assert d <= tol, d
    c.close()


def test_laplace_law_3d(gpu_lib):
    """Clean static sphere (beta = 0, no surfactant): the pressure jump
    settles near 2 sigma0/R (the 3D curvature and force normalisation).  As
    in 2D, W = 4 under-resolves |grad phi|^2 by ~7%, so the ratio sits near
    0.94; the 2D band [0.85, 1.02] applies (the unnormalised force would give
    1/6, a mean curvature of 1/R instead of 2/R one half)."""
    n, R, sigma0 = 48, 12.0, 1e-3
    phi, _ = W.drop_fields3(n, n, n, 24.3, 23.8, 24.1, R, 4.0)
    p = W.params3(nx=n, ny=n, nz=n, bc_y="periodic", flow="coupled", sigma0=sigma0, beta=0.0,
                  M_phi=0.05)
    c = ctx3(p, dict(phi=phi, c=np.zeros_like(phi)), "fp64")
    c.step(3000)
    f = c.read_fields(0)
    r = np.sqrt((np.arange(n)[None, None, :] - 24.3) ** 2 + (np.arange(n)[None, :, None] - 23.8) ** 2
                + (np.arange(n)[:, None, None] - 24.1) ** 2)
    dP = f["P"][r < R - 5].mean() - f["P"][r > R + 8].mean()
    print(f"Laplace 3D: dP = {dP:.4e}, 2 sigma/R = {2 * sigma0 / R:.4e}")
    assert 0.85 < dP / (2 * sigma0 / R) < 1.02
    c.close()


def test_sphere_surface_diffusion_l1(gpu_lib):
    """c_hat = (1 - cos theta)/2 on a static sphere: the l = 1 mode decays as
    exp(-l(l+1) D_s t/R^2) = exp(-2 D_s t/R^2)."""
    n, R, D = 64, 20.0, 0.1
    p, fl = W.static_drop3(n=n, R=R, D_s=D, center=(32.3, 31.8, 32.1))
    c = ctx3(p, fl, "fp64")
    x = np.arange(n)[None, None, :] - 32.3
    y = np.arange(n)[None, :, None] - 31.8
    z = np.arange(n)[:, None, None] - 32.1
    ct = x / np.sqrt(x * x + y * y + z * z)

    def amp(cc):
        return (cc * ct).sum() / cc.sum()

    a0 = amp(c.read_fields(0)["c"])
    steps = 1000
    c.step(steps)
    a1 = amp(c.read_fields(0)["c"])
    measured = -math.log(a1 / a0)
    expected = 2 * D * steps / R ** 2
    print(f"sphere l=1: measured {measured:.4f} expected {expected:.4f}")
    assert abs(measured / expected - 1) < 0.05
    c.close()


def test_c5_5000_steps_reduced_precision_tracks_fp64(gpu_lib):
    """The C5 configuration (256 x 128 x 128 coupled drop in shear, R = 32,
    Ca = 0.3, E = 0.2, c0 = 0.3, Re = 0.1) over its 5000 steps: no fault,
    phi and c conserved, and the FP32 and FP16 storage forms stay near the
    FP64 one.  The bound is loose because the problem is: inside the drop phi
    sits at 1 + 2e-5, where the sharpening flux amplifies rounding-level
    structure by ~0.7% per step (an FP64 run from phi perturbed by 1e-16
    moves by 1.1e-6 relative after 2000 steps, the same 2D drop by 6e-9), so
    FP32's 1e-7 storage rounding grows to O(1e-4) in phi and O(1e-3) in the
    small bulk surfactant values; the 2D C3 drop behaves alike (c: 2.9e-3
    after 5000 steps).  A wrong term moves the fields by orders more.  The
    same set-up scaled down by four is checked against the oracle's own
    FP32-storage and 2^-24 envelopes at 1000 and 5000 steps
    (test_gpu_long_horizon.py), where phi and c land at 1.0-1.1 x them;
    measured here: FP32 phi 4.7e-4, c 2.4e-3, u 1.2e-5; FP16 phi 8.9e-4,
    c 1.0e-2, u 1.8e-4.
    FP16 storage rounds stochastically; with random words hashed from the
    (node, step) pair its inventories only random-walk (1e-5 after 5000
    steps; 4.2M nodes put one standard deviation near 1e-4), where a seed
    that XORs a node hash with a step hash drifted phi by 2.9e-3."""
    p, fl = W.shear_drop3()
    out = {}
    for prec in ("fp64", "fp32", "fp16"):
        c = ctx3(p, fl, prec)
        s0 = c.inventory(0)
        c.step(5000)
        s1 = c.inventory(0)
        assert c.fault_flags(0) == 0
        drift = [abs(a - b) / abs(b) for a, b in zip(s1, s0)]
        print(prec, "inventory drift phi, c:", [f"{d:.1e}" for d in drift], flush=True)
        bound = {"fp64": (1e-13, 1e-12), "fp32": (1e-5, 1e-4), "fp16": (5e-4, 5e-4)}[prec]
        assert drift[0] < bound[0] and drift[1] < bound[1], (prec, drift)
        out[prec] = c.read_fields(0)
        c.close()
    b = out["fp64"]
    ub = np.stack([b["ux"], b["uy"], b["uz"]])
    for prec in ("fp32", "fp16"):
        a = out[prec]
        err = {k: float(np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k])) for k in ("phi", "c")}
        ua = np.stack([a["ux"], a["uy"], a["uz"]])
        err["u"] = float(np.linalg.norm(ua - ub) / np.linalg.norm(ub))
        print(f"C5 5000 steps, {prec} vs FP64:", {k: f"{v:.2e}" for k, v in err.items()},
              flush=True)
        if prec == "fp32":
            assert err["phi"] < 3e-3 and err["c"] < 2e-2 and err["u"] < 1e-3
        else:
            assert err["phi"] < 1e-2 and err["c"] < 5e-2 and err["u"] < 2e-3
