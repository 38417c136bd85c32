"""The 3D FP64 parity cases are well conditioned: a 1e-16 relative
perturbation of phi moves the oracle's own fields by well under 1e-12."""
import numpy as np
import pytest

from parity_cases3 import CASES3


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


@pytest.mark.parametrize("name", list(CASES3))
def test_parity_case3_is_well_conditioned(oracle_mod, name):
    build, steps = CASES3[name]
    p, fl = build()
    rng = np.random.default_rng(1)
    runs = []
    for eps in (0.0, 1e-16):
        phi = fl["phi"] * (1 + eps * rng.standard_normal(fl["phi"].shape))
        o = oracle_mod.OracleSim3(oracle_mod.make_params3(**p), phi, fl["c"], fl.get("ux"),
                                  fl.get("uy"), fl.get("uz"), fl.get("P"))
        assert o.run(steps) == 0
        runs.append(o.fields())
    a, b = runs
    for k in ("phi", "c"):
        assert _rel(b[k], a[k]) < 1e-13, (name, k)
    if p["flow"] != "none":
        u = lambda r: np.stack([r["ux"], r["uy"], r["uz"]])
        assert _rel(u(b), u(a)) < 1e-13, (name, "u")


@pytest.mark.parametrize("name", ["static3", "shear3", "density3"])
def test_fp16_parity_case3_damps_a_storage_rounding(oracle_mod, name):
    """The 3D FP16 parity cases keep a one-time relative perturbation of phi
    by one FP16 rounding (2.4e-4) below its own size over the run, so that
    the 1e-3 bar measures the storage."""
    build, steps = CASES3[name]
    p, fl = build()
    rng = np.random.default_rng(1)
    runs = []
    for eps in (0.0, 2.4e-4):
        phi = fl["phi"] * (1 + eps * rng.standard_normal(fl["phi"].shape))
        o = oracle_mod.OracleSim3(oracle_mod.make_params3(**p), phi, fl["c"], fl.get("ux"),
                                  fl.get("uy"), fl.get("uz"), fl.get("P"))
        assert o.run(steps) == 0
        runs.append(o.fields())
    a, b = runs
    for k in ("phi", "c"):
        assert _rel(b[k], a[k]) < 2.4e-4, (name, k, _rel(b[k], a[k]))
