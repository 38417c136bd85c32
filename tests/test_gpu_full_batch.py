"""The benchmark's own workloads at full size, in the launch configurations
the benchmark times, against the FP64 oracle run at full size from the same
fields.

2D: the 64 seeded coupled shear drops (default_rng(2504); 18,399,232 nodes,
grids 256 x 256 to 1024 x 512), set up by bench.make_ctx on a dedicated
stream and advanced STEPS steps through HIP graphs, one launch per step for
all 64 simulations: FP32 autotuned as the benchmark's headline run does (the
library keeps the fastest tile shape and store policy), FP64 and FP16 with
the default launch the benchmark's other storage forms use.  Every
simulation is compared with the oracle.

3D: the 256 x 128 x 128 coupled drop (4,194,304 nodes) set up by
bench.make_ctx3 (default collision columns and store policy) in every
precision, against one oracle run.

Tolerances are those of the parity tests: relative L2 on phi, c and u of
1e-12 (FP64), 1e-5 (FP32) and 1e-3 (FP16 storage)."""
import os
import sys

import numpy as np
import pytest

from paper_2504_09024_amd import workloads as W
from parity_util import field_errors, oracle_sim, rel_l2

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

pytestmark = pytest.mark.gpu

STEPS = 20   # one full graph of 16 steps plus a partial one
STEPS3 = 4
TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp16": 1e-3}


@pytest.fixture(scope="module")
def batch():
    sims = W.batched_shear_drops(64)
    assert bench.nodes_of(sims) == 18_399_232
    return sims


@pytest.fixture(scope="module")
def batch_oracle(oracle_mod, batch):
    out = []
    for p, fl in batch:
        o = oracle_sim(oracle_mod, p, fl)
        assert o.run(STEPS) == 0
        out.append(o.fields())
    return out


def _on_stream(fn):
    import torch
    tstream = torch.cuda.Stream()
    torch.cuda.set_stream(tstream)
    try:
        return fn(tstream.cuda_stream)
    finally:
        torch.cuda.set_stream(torch.cuda.default_stream())


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp16"])
def test_full_batch_in_bench_configuration(gpu_lib, batch, batch_oracle, prec):
    from paper_2504_09024_amd import cmlb

    def run(stream):
        ctx = bench.make_ctx(cmlb, batch, prec, stream)
        if prec == "fp32":
            width, rows, stores = ctx.autotune(20)
            print(f"autotuned launch {width}x{rows}, {stores} stores", flush=True)
        assert ctx.step_count == 0
        ctx.step(STEPS)
        assert ctx.step_count == STEPS
        fields = [ctx.read_fields(i) for i in range(len(batch))]
        assert all(ctx.fault_flags(i) == 0 for i in range(len(batch)))
        ctx.close()
        return fields

    fields = _on_stream(run)
    worst = {}
    for i, (p, _) in enumerate(batch):
        err = field_errors(fields[i], batch_oracle[i], True, True)
        for k in ("phi", "c", "u"):
            worst[k] = max(worst.get(k, 0.0), err[k])
    print(f"{prec} worst over 64 sims:", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    for k, v in worst.items():
        assert np.isfinite(v) and v <= TOL[prec], (k, v)


@pytest.fixture(scope="module")
def drop3(oracle_mod):
    p, fl = W.shear_drop3()
    assert p["nx"] * p["ny"] * p["nz"] == 4_194_304
    o = oracle_mod.OracleSim3(oracle_mod.make_params3(**p), fl["phi"], fl["c"], fl["ux"],
                              fl["uy"], fl["uz"])
    assert o.run(STEPS3) == 0
    return p, fl, o.fields()


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp16"])
def test_full_c5_in_bench_configuration(gpu_lib, drop3, prec):
    from paper_2504_09024_amd import cmlb
    p, fl, of = drop3

    def run(stream):
        ctx = bench.make_ctx3(cmlb, [(p, fl)], prec, stream)
        ctx.step(STEPS3)
        g = ctx.read_fields(0)
        assert ctx.fault_flags(0) == 0
        ctx.close()
        return g

    g = _on_stream(run)
    err = {"phi": rel_l2(g["phi"], of["phi"]), "c": rel_l2(g["c"], of["c"]),
           "u": rel_l2(np.stack([g["ux"], g["uy"], g["uz"]]),
                       np.stack([of["ux"], of["uy"], of["uz"]]))}
    print(f"C5 {prec} {STEPS3} steps:", {k: f"{v:.2e}" for k, v in err.items()}, flush=True)
    for k, v in err.items():
        assert np.isfinite(v) and v <= TOL[prec], (k, v)
