"""The FP64 parity bar (1e-12 relative L2) is only meaningful where the
problem itself is well conditioned: a relative perturbation of 1e-16 on phi
(one rounding) must move the oracle's own fields by well under 1e-12 over
the same number of steps.  Cases whose drop centre sits on a node with
theta > eps (the regularised normal of Eq. CACE is then anti-diffusive
there) fail this check and are not used as FP64 parity cases."""
import numpy as np
import pytest

from parity_cases import CASES, FP16_CONDITIONING, FP16_FIELDS, FP64_CONDITIONING
from parity_util import field_errors, oracle_sim
from paper_2504_09024_amd import workloads as W


def _perturbed(fl, eps, seed=1):
    rng = np.random.default_rng(seed)
    out = dict(fl)
    out["phi"] = fl["phi"] * (1 + eps * rng.standard_normal(fl["phi"].shape))
    return out


def _sensitivity(oracle, p, fl, steps, eps=1e-16):
    a = oracle_sim(oracle, p, fl)
    b = oracle_sim(oracle, p, _perturbed(fl, eps))
    a.run(steps)
    b.run(steps)
    fa, fb = a.fields(), b.fields()
    flow = p["flow"]
    return field_errors(fb, fa, flow == "coupled", flow != "none")


@pytest.mark.parametrize("name", FP64_CONDITIONING)
def test_parity_case_is_well_conditioned(oracle_mod, name):
    build, steps = CASES[name]
    p, fl = build()
    err = _sensitivity(oracle_mod, p, fl, steps)
    for k in ("phi", "c", "u", "P"):
        if k in err:
            assert err[k] < 1e-13, (name, k, err[k])


def test_node_centred_small_drop_is_ill_conditioned(oracle_mod):
    """Counter-example: R/W = 4 with the centre on a node (theta = 1e-7 where
    grad phi = 0) amplifies the 1e-16 perturbation by many orders."""
    p, fl = W.static_drop(n=64, R=16.0)
    err = _sensitivity(oracle_mod, p, fl, 100)
    assert err["phi"] > 1e-11


@pytest.mark.parametrize("name,steps", FP16_CONDITIONING)
def test_fp16_parity_case_damps_a_storage_rounding(oracle_mod, name, steps):
    """The FP16 bar (1e-3) measures the storage only where one FP16-sized
    rounding of phi (2.4e-4 relative) does not grow over the run."""
    build, _ = CASES[name]
    p, fl = build()
    err = _sensitivity(oracle_mod, p, fl, steps, eps=2.4e-4)
    for k in FP16_FIELDS.get(name, ("phi", "c", "u")):
        if k in err:
            assert err[k] < 2.4e-4, (name, k, err[k])


def test_random_fields_amplify_an_fp16_rounding(oracle_mod):
    """Counter-example kept out of the FP16 parity cases: the random O(1)
    fields of coupled_random turn the same perturbation into 2.6e-2 of phi
    after 150 steps (x 100), where FP32's rounding still stays far below its
    bar."""
    build, steps = CASES["coupled_random"]
    p, fl = build()
    err = _sensitivity(oracle_mod, p, fl, steps, eps=2.4e-4)
    assert err["phi"] > 1e-2
