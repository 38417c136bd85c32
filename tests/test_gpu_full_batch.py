"""The benchmark's own workload at full size, in the launch configuration the
benchmark times, against the FP64 oracle.

The 64 seeded coupled shear drops (default_rng(2504); 18,399,232 nodes, grids
256 x 256 to 1024 x 512) are set up in FP32 by bench.make_ctx on a dedicated
stream, autotuned as the benchmark does (the library keeps the fastest tile
shape and store policy), and advanced STEPS steps through HIP graphs, one
launch per step for all 64 simulations.  Every simulation is then compared
with the oracle run at its full size from the same fields, to the FP32
tolerance of the parity tests (relative L2 <= 1e-5 on phi, c and u)."""
import os
import sys

import numpy as np
import pytest

from paper_2504_09024_amd import workloads as W
from parity_util import field_errors, oracle_sim

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

pytestmark = pytest.mark.gpu

STEPS = 20  # one full graph of 16 steps plus a partial one
TOL = 1e-5


def test_full_batch_in_bench_configuration(oracle_mod, gpu_lib):
    import torch
    from paper_2504_09024_amd import cmlb
    sims = W.batched_shear_drops(64)
    assert bench.nodes_of(sims) == 18_399_232
    tstream = torch.cuda.Stream()
    torch.cuda.set_stream(tstream)
    try:
        ctx = bench.make_ctx(cmlb, sims, "fp32", tstream.cuda_stream)
        width, rows, stores = ctx.autotune(20)
        print(f"autotuned launch {width}x{rows}, {stores} stores", flush=True)
        assert ctx.step_count == 0
        ctx.step(STEPS)
        assert ctx.step_count == STEPS
        fields = [ctx.read_fields(i) for i in range(len(sims))]
        assert all(ctx.fault_flags(i) == 0 for i in range(len(sims)))
        ctx.close()
    finally:
        torch.cuda.set_stream(torch.cuda.default_stream())
    worst = {}
    for i, (p, fl) in enumerate(sims):
        o = oracle_sim(oracle_mod, p, fl)
        assert o.run(STEPS) == 0
        err = field_errors(fields[i], o.fields(), True, True)
        for k in ("phi", "c", "u"):
            worst[k] = max(worst.get(k, 0.0), err[k])
        if i % 16 == 0:
            print(f"sim {i} {p['nx']}x{p['ny']}:", {k: f"{err[k]:.2e}" for k in ("phi", "c", "u")},
                  flush=True)
    print("worst over 64 sims:", {k: f"{v:.2e}" for k, v in worst.items()}, flush=True)
    for k, v in worst.items():
        assert np.isfinite(v) and v <= TOL, (k, v)
