#!/usr/bin/env python3
"""Throughput of the coupled central-moment LB step on one MI355X.

Default workload: the coupled surfactant-laden shear drop of Sec. 4.3 scaled
to 1024 x 512 (R = 64, Ca = 0.3, E = 0.2, c0/c_max = 0.3, Re = 0.1), FP32
storage and arithmetic.  A step is one collide-and-stream pass of all three
lattices over every node; populations stay resident in HBM.  Prints one JSON
line: coupled MLUPS, the dominant kernel's roofline fraction (algorithmic
bytes over HIP-event-timed launches on the kernel's stream), the other
storage forms and the batched form, and the CPU oracle timed on a bounded
sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled MLUPS and % HBM roofline, FP32/FP16-storage/batched vs FP64 GPU"
HBM_PEAK_GBS = 8000.0
STORAGE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}
ARITH = {"fp64": "f64", "fp32": "f32", "fp16": "f32"}
KERNEL_SOURCES = ("paper_2504_09024_amd/csrc/kernels.hpp", "paper_2504_09024_amd/csrc/lattice.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes_per_node(prec, lattices=3):
    """Every population read once and written once per step."""
    return lattices * 9 * 2 * STORAGE_BYTES[prec]


def kernel_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def timed_run(ctx, steps, warmup, torch):
    """Warm up, then time exactly `steps` steps with HIP events on the stream
    the library launches on (torch's current stream)."""
    ctx.step(warmup)
    ctx.synchronize()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    ctx.step(steps)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.synchronize()
    return start.elapsed_time(end) / 1e3, wall


def make_ctx(cmlb, sims, prec, stream):
    ps = [s[0] for s in sims]
    ctx = cmlb.Context(ps, prec, stream=stream)
    for i, (_, fl) in enumerate(sims):
        ctx.init_fields(i, fl["phi"], fl["c"], fl.get("ux"), fl.get("uy"), fl.get("P"))
    return ctx


def traffic_entry(workload_key, prec):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = data.get(f"{workload_key}:{prec}")
    if not ent or ent.get("kernel_hash") != kernel_hash():
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(p, fl, steps):
    import oracle
    o = oracle.OracleSim(oracle.make_params(**p), fl["phi"], fl["c"], fl.get("ux"),
                         fl.get("uy"), fl.get("P"))
    t0 = time.perf_counter()
    o.run(steps)
    dt = time.perf_counter() - t0
    nodes = p["nx"] * p["ny"]
    return {"value": nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} steps of the full {p['nx']}x{p['ny']} coupled grid "
                      f"({dt:.1f} s, FP64, OpenMP over rows)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16"])
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the other storage forms")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=24)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
              "multi-GPU sharding is a design note, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_09024_amd import cmlb
    from paper_2504_09024_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    # a dedicated stream (default priority): the library launches on it and
    # torch's events are recorded on it
    tstream = torch.cuda.Stream()
    torch.cuda.set_stream(tstream)
    stream = tstream.cuda_stream

    p, fl = W.shear_drop()
    nodes = p["nx"] * p["ny"]
    prec = args.precision
    log(f"[bench] workload C3 1024x512 coupled, {prec}, warmup {args.warmup}, steps {args.steps}")
    ctx = make_ctx(cmlb, [(p, fl)], prec, stream)
    if args.tile_rows:
        ctx.set_tile_rows(args.tile_rows)
    ctx.set_use_graph(not args.no_graph)
    gpu_s, wall_s = timed_run(ctx, args.steps, args.warmup, torch)
    inv = ctx.inventory(0)
    ctx.close()
    mlups = nodes * args.steps / gpu_s / 1e6
    ms_per_step = gpu_s * 1e3 / args.steps
    bpl = algorithmic_bytes_per_node(prec) * nodes
    achieved = bpl / (gpu_s / args.steps) / 1e9
    log(f"[bench] {mlups:.0f} MLUPS, {ms_per_step * 1e3:.2f} us/step, {achieved:.0f} GB/s "
        f"(wall {wall_s:.3f} s)")

    forms = {}
    if not args.no_forms:
        for fp in ("fp64", "fp32", "fp16"):
            if fp == prec:
                forms[fp] = {"MLUPS": round(mlups, 1)}
                continue
            c2 = make_ctx(cmlb, [(p, fl)], fp, stream)
            k = max(200, args.steps // 4)
            s, _ = timed_run(c2, k, 50, torch)
            c2.close()
            forms[fp] = {"MLUPS": round(nodes * k / s / 1e6, 1)}
            log(f"[bench] form {fp}: {forms[fp]['MLUPS']} MLUPS")
        sims = W.batched_shear_drops(64)
        bnodes = sum(s[0]["nx"] * s[0]["ny"] for s in sims)
        for fp in ("fp32", "fp16"):
            c3 = make_ctx(cmlb, sims, fp, stream)
            k = 100
            s, _ = timed_run(c3, k, 10, torch)
            c3.close()
            forms[f"batched64_{fp}"] = {
                "MLUPS": round(bnodes * k / s / 1e6, 1), "nodes": bnodes,
                "hbm_frac": round(algorithmic_bytes_per_node(fp) * bnodes / (s / k) / 1e9
                                  / HBM_PEAK_GBS, 3)}
            log(f"[bench] batched64 {fp}: {forms[f'batched64_{fp}']}")
        base = forms["fp64"]["MLUPS"]
        for v in forms.values():
            v["speedup_vs_fp64_gpu"] = round(v["MLUPS"] / base, 2)

    cpu = None
    if not args.no_cpu:
        log(f"[bench] CPU oracle sample: {args.cpu_steps} steps")
        cpu = cpu_baseline(p, fl, args.cpu_steps)

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ARITH[prec],
        "data": "synthetic",
        "config": {
            "workload": "coupled surfactant-laden shear drop, 1024x512, R=64, Ca=0.3, E=0.2, "
                        "c0/c_max=0.3, Re=0.1, walls at +-U0",
            "nx": p["nx"], "ny": p["ny"], "nodes": nodes, "storage": prec,
            "lattices": 3, "graph": not args.no_graph,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_entry("c3", prec),
        },
        "cpu_baseline": cpu,
        "forms": forms,
        "inventory": {"phi": inv[0], "c": inv[1]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
