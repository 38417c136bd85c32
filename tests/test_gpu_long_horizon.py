"""Reduced precision over the full horizons of the long workloads, at full
size, bounded by how strongly the problem itself amplifies FP32-scale
perturbations.

The bounds come from tests/golden/sensitivity.json, which the FP64 oracle
alone writes (tests/golden/make_sensitivity.py): for each workload the
relative L2 difference between the oracle and the same oracle with every
stored population rounded to FP32 after each step ("fp32": FP32 storage
rounding alone, arithmetic left in FP64), and with phi perturbed once by
2^-24 ("perturbed").  The envelope of a field is the larger of the two.

The GPU's FP32 form also computes in FP32 (moments, stencils, forces,
collisions).  On phi and c that adds rounding of the same order as the
storage: the FP32 form lands at 0.6-4.7 x the envelope, bounded here by
K_FIELDS = 5.  The velocity of the shear drops lands at 0.4, 1.5 and 1.7 x
the envelope after 5000 steps (Ca = 0.1, 0.3, 0.5) and that of the 3D
scale-down at 5.3 x after 1000 steps, bounded by K_U = 8.  Four systematic
FP32 biases of the flow lattice were removed on the way there: the velocity
decode and the first raw moments use the same FP32 value of rho cs^2; the
collision changes the momentum by exactly cs^2 F instead of re-encoding it
from the rounded u; the lattice weights and the rest value rho_b/9 of the
third-order moments enter through correctly rounded divisions instead of
products with the rounded 1/9 (these two took the wall slip of the
Ca = 0.5 drop from 1.2e-5 to 2e-7 of the wall speed and its velocity error
from 32 x to 12.8 x the envelope); and the map from the flow lattice's
post-collision moments back to populations runs in FP64, so the stored
values carry only the rounding of the store (12.8 x to 1.7 x; the FP32 sums
of that map rounded alike every step at a quasi-steady node and left a
steady momentum error).  In 3D the equilibrium's departure from the rest
moments is built without the cancellation cs2 - (cs2 + u^2).

Also here: one step of the oracle from the GPU's own state after the full
horizon, which checks the step itself at a late, developed state (FP64 to
1e-13, FP32 to 1e-6 of the largest population).
"""
import json
import os

import numpy as np
import pytest

from paper_2504_09024_amd import workloads as W
from parity_util import field_errors, gpu_ctx

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "golden", "sensitivity.json")) as _fh:
    GOLD = json.load(_fh)

K_FIELDS = 5.0
K_U = 8.0


def envelope(env, k):
    """The larger of the storage-rounding and the one-time envelopes of
    field k (None where the field is zero)."""
    vals = [env[v].get(k) for v in ("fp32", "perturbed")]
    vals = [v for v in vals if v is not None]
    return max(vals) if vals else None


def _check_envelope(err, env, label, k_fields=K_FIELDS, k_u=K_U):
    """err: GPU FP32-vs-FP64 (or -vs-oracle) relative L2 per field; env:
    the oracle's envelopes at the same step."""
    for k, v in err.items():
        e = envelope(env, k)
        if e is None:
            continue
        kk = k_u if k == "u" else k_fields
        print(f"{label} {k}: FP32 {v:.2e}, envelope {e:.2e} (x{v / e:.2f}; storage "
              f"{env['fp32'][k]:.2e}, one-time {env['perturbed'][k]:.2e})", flush=True)
        assert v <= kk * e, (label, k, v, e)


def _gpu_fields(ctx):
    return ctx.read_fields(0)


@pytest.mark.parametrize("ca", [0.1, 0.3, 0.5])
def test_c3_fp32_within_envelope_1000_and_5000_steps(gpu_lib, ca):
    """C3: the coupled shear drop at full size (1024x512, Re = 0.1, E = 0.2,
    c0 = 0.3, Sec. 4.3 set-up), FP32 against FP64 after 1000 and 5000
    steps."""
    key = f"c3_Ca{ca}"
    if key not in GOLD:
        pytest.skip(f"envelope {key} not generated yet (tests/golden/make_sensitivity.py)")
    p, fl = W.shear_drop(Ca=ca)
    c64 = gpu_ctx(p, fl, "fp64")
    c32 = gpu_ctx(p, fl, "fp32")
    t = 0
    for t_end in (1000, 5000):
        c64.step(t_end - t)
        c32.step(t_end - t)
        t = t_end
        g64, g32 = _gpu_fields(c64), _gpu_fields(c32)
        err = field_errors(g32, g64, True, True)
        err = {k: err[k] for k in ("phi", "c", "u")}
        _check_envelope(err, GOLD[key][str(t_end)], f"{key} t={t_end}")
    # conservation over the horizon: FP64 to rounding; FP32 drifts by
    # 1.0-1.1e-5 in phi and 0.3-4e-7 in c over 5000 steps (the oracle with
    # FP32 storage rounding alone: at most 6e-7 and 8e-7), reported and
    # bounded at 3e-5
    i64 = np.array(c64.inventory(0))
    i32 = np.array(c32.inventory(0))
    o = np.array([fl["phi"].sum(), fl["c"].sum()])
    print(key, "drift FP64", np.abs(i64 - o) / o, "FP32", np.abs(i32 - o) / o)
    assert np.all(np.abs(i64 - o) <= 1e-12 * o)
    assert np.all(np.abs(i32 - o) <= 3e-5 * o)
    c64.close()
    c32.close()


def test_c2_fp32_within_envelope_full_period(gpu_lib):
    """C2: the drop in the time-reversing vortex (512x512, R = 64, T = 20000),
    FP32 against FP64 at T/4, T/2 and T."""
    p, fl = W.vortex_drop()
    c64 = gpu_ctx(p, fl, "fp64")
    c32 = gpu_ctx(p, fl, "fp32")
    t = 0
    for t_end in (5000, 10000, 20000):
        c64.step(t_end - t)
        c32.step(t_end - t)
        t = t_end
        err = field_errors(_gpu_fields(c32), _gpu_fields(c64), False, True)
        _check_envelope({k: err[k] for k in ("phi", "c")}, GOLD["c2"][str(t_end)],
                        f"c2 t={t_end}")
    c64.close()
    c32.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-6)])
def test_c3_one_step_from_gpu_state_after_5000(oracle_mod, gpu_lib, prec, tol):
    """After 5000 steps of C3 (Ca = 0.3), one oracle step from the GPU's own
    populations against the GPU's next step, relative to the largest
    population of each lattice.  By then c is negative inside the drop
    (about -7e-3 at its centre, the drift of the surfactant out of a bulk
    whose phi over- and undershoots), where |grad phi| is 1e-7 and the
    regularised normal grad phi / (|grad phi| + 1e-12) points wherever the
    rounding of phi points: there the confining flux D_s theta_c n of h
    depends on the order of summation (FP64: 1.3e-12 of the largest h;
    FP32: 9e-4).  h is therefore compared where the normal is defined by
    phi rather than by its rounding: |grad phi| > 1e-6 in FP64 and > 1e-4 in
    FP32 (phi near 1 carries 6e-8 in FP32, so its gradient carries about
    3e-8); f and g everywhere (FP32: 2.6e-7 measured for f, 1.4e-10 for
    g)."""
    p, fl = W.shear_drop(Ca=0.3)
    ctx = gpu_ctx(p, fl, prec)
    ctx.step(5000)
    f, h, g = ctx.get_populations(0)
    phi = ctx.read_fields(0)["phi"]
    o = oracle_mod.OracleSim.from_populations(oracle_mod.make_params(**p), f, h, g, t=5000)
    assert o.run(1) == 0
    ctx.step(1)
    f1, h1, g1 = ctx.get_populations(0)
    ctx.close()
    gy, gx = np.gradient(phi)
    defined = (np.hypot(gx, gy) > (1e-6 if prec == "fp64" else 1e-4))[None, :, :]
    for name, a, b in (("f", f1, o.f), ("h", h1, o.h), ("g", g1, o.g)):
        d = np.abs(a - b)
        d_all = d.max() / np.abs(b).max()
        if name == "h":
            d = d * defined
        dm = d.max() / np.abs(b).max()
        print(f"C3 {prec} one step after 5000, {name}: {dm:.2e} (everywhere {d_all:.2e})")
        assert dm <= tol, (name, dm)


def test_c5_scaled_fp32_within_envelope_1000_and_5000_steps(gpu_lib):
    """The 3D drop in shear (C5 set-up) scaled down by four in every
    direction, 64 x 32 x 32 with R = 8, FP32 against FP64 after 1000 and
    5000 steps, against the 3D oracle's own envelopes at that size (the
    full-size run is beyond the CPU oracle's reach at these horizons).
    Measured: phi 1.05 x and c 1.03 x the envelope at 1000 steps, 1.0 x
    both at 5000; u 5.3 x at 1000 and 0.92 x at 5000.  The 3D flow collision uses
    the 2D remedies (weights through correctly rounded divisions by 27, the
    exact momentum change), which took the sheared bulk's mean velocity
    profile error from 3.7e-6 to 6e-8 of U0, and forms the equilibrium's
    departure from the rest moments without the cancellation
    cs2 - (cs2 + u^2), which took u from 1.3e-5 (1000 steps) to 1.5e-7."""
    from paper_2504_09024_amd import cmlb
    key = "c5_64x32x32"
    if key not in GOLD:
        pytest.skip(f"envelope {key} not generated yet (tests/golden/make_sensitivity.py)")
    p, fl = W.shear_drop3(nx=64, ny=32, nz=32, R=8.0)
    ctx = {}
    for prec in ("fp64", "fp32"):
        c = cmlb.Context3([p], prec)
        c.init_fields(0, fl["phi"], fl["c"], fl.get("ux"), fl.get("uy"), fl.get("uz"), fl.get("P"))
        ctx[prec] = c
    t = 0
    for t_end in (1000, 5000):
        for c in ctx.values():
            c.step(t_end - t)
        t = t_end
        a, b = ctx["fp32"].read_fields(0), ctx["fp64"].read_fields(0)
        rel = lambda x, y: float(np.linalg.norm(x - y) / np.linalg.norm(y))
        u = lambda r: np.stack([r["ux"], r["uy"], r["uz"]])
        env = GOLD[key][str(t_end)]
        _check_envelope({"phi": rel(a["phi"], b["phi"]), "c": rel(a["c"], b["c"])}, env,
                        f"{key} t={t_end}")
        eu = rel(u(a), u(b))
        bound = K_U * envelope(env, "u")
        print(f"{key} t={t_end} u: FP32 {eu:.2e}, envelope {envelope(env, 'u'):.2e}, "
              f"bound {bound:.2e}", flush=True)
        assert eu <= bound, (t_end, eu, bound)
    for c in ctx.values():
        assert c.fault_flags(0) == 0
        c.close()
