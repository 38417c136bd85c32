"""The sensitivity envelopes that bound the long-horizon FP32 checks
(tests/golden/sensitivity.json) are reproducible, and they measure the
problem, not the arithmetic: CPU only, FP64 oracle.

The cheap entries are recomputed here with the committed generator and must
match the stored values (the oracle is deterministic whatever its thread
count).  The scale-down of the C3 shear drop also shows the amplification
itself: a one-time relative perturbation of phi by 2^-24 grows about
thirty-fold in 1000 steps (the sharpening flux acting on rounding-level
structure inside the drop), so FP32-scale differences at long horizons are a
property of the problem at FP32 scale.
"""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_sensitivity as MS  # noqa: E402

with open(os.path.join(HERE, "golden", "sensitivity.json")) as _fh:
    GOLD = json.load(_fh)


def _close(a, b):
    for t, per in b.items():
        for variant, fields in per.items():
            for k, v in fields.items():
                got = a[t][variant][k]
                if v is None:
                    assert got is None, (t, variant, k, got)
                else:
                    assert abs(got - v) <= 1e-9 * abs(v), (t, variant, k, got, v)


@pytest.mark.parametrize("key", ["coupled_random", "c3_256x128_Ca0.3"])
def test_stored_envelope_is_reproduced(oracle_mod, tmp_path, key):
    builder, checkpoints = MS.workloads()[key]
    got = MS.sensitivity(key, builder, checkpoints, str(tmp_path))
    _close(got, GOLD[key])


def test_c3_scale_down_amplifies_a_one_time_fp32_perturbation():
    """The stored C3 scale-down entry: after 1000 steps the one-time 2^-24
    perturbation of phi has grown to 2e-6 in phi and 3e-5 in c (relative
    L2), far above the 6e-8 it started at."""
    e = GOLD["c3_256x128_Ca0.3"]["1000"]["perturbed"]
    assert e["phi"] > 10 * 2.0 ** -24
    assert e["c"] > 100 * 2.0 ** -24


def test_every_long_horizon_workload_has_its_envelope():
    """Each workload and checkpoint that the long-horizon GPU checks use has
    a stored envelope, positive for phi and c in both variants."""
    need = {"c1": (500, 2000), "coupled_random": (150,), "c2": (5000, 10000, 20000),
            "c3_Ca0.1": (1000, 5000), "c3_Ca0.3": (1000, 5000), "c3_Ca0.5": (1000, 5000),
            "c5_64x32x32": (1000, 5000)}
    for key, ts in need.items():
        for t in ts:
            for variant in ("fp32", "perturbed"):
                e = GOLD[key][str(t)][variant]
                assert e["phi"] > 0 and e["c"] > 0, (key, t, variant, e)
