#!/usr/bin/env python3
"""Throughput of the coupled central-moment LB step on one MI355X.

Headline workload: 64 independent coupled surfactant-laden shear drops
(Sec. 4.3 set-up) with seeded sizes from 256x256 to 1024x512 and seeded
Ca, E, c0/c_max, Pe_s (numpy default_rng(2504)), advanced together by one
launch per step; FP32 storage and arithmetic; 18.4 M nodes, 4 GB of
populations (double-buffered), far above the 256 MB Infinity Cache, so HBM
is the bound.  A step is one collide-and-stream pass of all three lattices
over every node of every simulation; populations stay resident in HBM.

Prints one JSON line: coupled MLUPS, the step kernel's roofline fraction
(algorithmic bytes over HIP-event-timed launches on the kernel's stream),
the plain-copy ceiling measured in the same run (the library's copy with
non-temporal loads and stores, 2 GiB buffers; also with the buffers split
into 27 planes copied side by side, the step's own number of streams) and
the step's fraction of it,
the other storage forms (FP64, FP16) of the batch, of the single 1024x512
drop and of the 3D drop, and the CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32]
                       [--workload batched|c3]
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
# sources whose change invalidates counter-measured traffic (the build
# flags included), per lattice dimension
KERNEL_SOURCES = {
    2: ("paper_2504_09024_amd/csrc/kernels.hpp", "paper_2504_09024_amd/csrc/lattice.hpp",
        "paper_2504_09024_amd/csrc/device_common.hpp", "paper_2504_09024_amd/build.py"),
    3: ("paper_2504_09024_amd/csrc/kernels3.hpp", "paper_2504_09024_amd/csrc/device_common.hpp",
        "paper_2504_09024_amd/build.py"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes_per_node(prec, lattices=3, q=9):
    """Every population read once and written once per step (q = 9 for
    D2Q9, 27 for D3Q27)."""
    return lattices * q * 2 * STORAGE_BYTES[prec]


def kernel_hash(dim=2):
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[dim]:
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


def make_ctx3(cmlb, sims, prec, stream, graph=True, shape=None, stores="auto"):
    ctx = cmlb.Context3([s[0] for s in sims], prec, stream=stream)
    ctx.set_use_graph(graph)
    ctx.set_store_policy(stores)
    if shape:
        ctx.set_tile_shape(*shape)
    for i, (_, fl) in enumerate(sims):
        ctx.init_fields(i, fl["phi"], fl["c"], fl.get("ux"), fl.get("uy"), fl.get("uz"),
                        fl.get("P"))
    return ctx


def make_ctx(cmlb, sims, prec, stream, tile_rows=0, graph=True, xcd_remap=True, group=-1,
             stores="auto", tile_width=0):
    ps = [s[0] for s in sims]
    ctx = cmlb.Context(ps, prec, stream=stream)
    if tile_rows:
        ctx.set_tile_shape(tile_width or 64, tile_rows)
    ctx.set_store_policy(stores)
    if group >= 0:
        ctx.set_tile_order(group)
    ctx.set_use_graph(graph)
    ctx.set_xcd_remap(xcd_remap)
    for i, (_, fl) in enumerate(sims):
        ctx.init_fields(i, fl["phi"], fl["c"], fl.get("ux"), fl.get("uy"), fl.get("P"))
    return ctx


def traffic_entry(workload_key, prec, dim=2):
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
    if not ent or ent.get("kernel_hash") != kernel_hash(dim):
        return None
    return ent.get("bytes_per_launch")


def _counter_kib(csv_path, counter, kernel_substr):
    """Mean per-dispatch value of `counter` over the dispatches of kernels
    whose name contains `kernel_substr` in a rocprofv3 counter_collection.csv
    (values of one dispatch summed over their instances)."""
    import csv
    per = {}
    with open(csv_path, newline="") as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter or kernel_substr not in r["Kernel_Name"]:
                continue
            per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    if not per:
        raise ValueError(f"no {counter} rows for '{kernel_substr}' in {csv_path}")
    return sum(per.values()) / len(per), len(per)


def record_traffic(key, nodes, prec, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv,
                   copy_bytes, path=None, lattices=3, q=9, kernels=("k_step",)):
    """Scale the step kernels' FETCH_SIZE / WRITE_SIZE (KiB per dispatch,
    summed over the kernels of one step: k_step in 2D, k_moments3 and
    k_collide3 in 3D) by what the same counters read for a plain device copy
    of copy_bytes, and store HBM bytes per step under `key` in
    profiles/traffic.json, tagged with the hash of the kernel sources."""
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    cf, _ = _counter_kib(copy_fetch_csv, "FETCH_SIZE", "copyBuffer")
    cw, _ = _counter_kib(copy_write_csv, "WRITE_SIZE", "copyBuffer")
    fetch_scale = copy_bytes / (cf * 1024.0)
    write_scale = copy_bytes / (cw * 1024.0)
    kf = kw = 0.0
    nf, nw, per_kernel = [], [], {}
    for kn in kernels:
        f1, n1 = _counter_kib(fetch_csv, "FETCH_SIZE", kn)
        w1, n2 = _counter_kib(write_csv, "WRITE_SIZE", kn)
        kf += f1
        kw += w1
        nf.append(n1)
        nw.append(n2)
        per_kernel[kn] = {"fetch_bytes": int(round(f1 * 1024.0 * fetch_scale)),
                          "write_bytes": int(round(w1 * 1024.0 * write_scale))}
    fetch = kf * 1024.0 * fetch_scale
    write = kw * 1024.0 * write_scale
    alg = algorithmic_bytes_per_node(prec, lattices, q) * nodes
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data["_note"] = ("HBM-side bytes per step (one step-kernel launch in 2D; the moments and "
                     "collision launches in 3D) from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE "
                     "(KiB per dispatch), each scaled by the counter's reading for a plain device "
                     "copy (bench.py --copy-calibration).")
    data["calibration"] = {"copy_bytes": copy_bytes, "FETCH_SIZE_KiB": round(cf, 2),
                           "WRITE_SIZE_KiB": round(cw, 2), "fetch_scale": fetch_scale,
                           "write_scale": write_scale}
    data[key] = {"kernel_hash": kernel_hash(3 if len(kernels) > 1 else 2),
                 "bytes_per_launch": int(round(fetch + write)),
                 "fetch_bytes": int(round(fetch)), "write_bytes": int(round(write)),
                 "algorithmic_bytes": alg,
                 "traffic_over_algorithmic": round((fetch + write) / alg, 4),
                 "fetch_over_algorithmic_reads": round(fetch / (alg / 2), 4),
                 "dispatches": [sum(nf), sum(nw)]}
    if len(kernels) > 1:
        data[key]["per_kernel"] = per_kernel
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1)
        fh.write("\n")
    return data[key]


def cpu_baseline(sims, target_s=12.0):
    """The FP64 oracle on a bounded sample of the workload: the first
    simulation of the set, as many steps as fit ~target_s (at least 2)."""
    import oracle
    p, fl = sims[0]
    if "nz" in p:
        o = oracle.OracleSim3(oracle.make_params3(**p), fl["phi"], fl["c"], fl.get("ux"),
                              fl.get("uy"), fl.get("uz"), fl.get("P"))
    else:
        o = oracle.OracleSim(oracle.make_params(**p), fl["phi"], fl["c"], fl.get("ux"),
                             fl.get("uy"), fl.get("P"))
    t0 = time.perf_counter()
    o.run(2)
    dt = time.perf_counter() - t0
    steps = 2
    # the first steps are slower (threads and pages warming up), so keep
    # going in chunks sized from the running rate until target_s is reached
    while dt < target_s and steps < 20000:
        n = min(20000 - steps, max(1, int((target_s - dt) * steps / dt) + 1))
        t1 = time.perf_counter()
        o.run(n)
        dt += time.perf_counter() - t1
        steps += n
    nodes = p["nx"] * p["ny"] * p.get("nz", 1)
    size = "x".join(str(p[k]) for k in ("nx", "ny", "nz") if k in p)
    return {"value": round(nodes * steps / dt / 1e6, 3), "unit": "MLUPS",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} steps of simulation 0 of the workload ({size} "
                      f"{p.get('flow', 'coupled')}, {dt:.1f} s, FP64, OpenMP over rows)"}


def oracle_leg(name, min_s=2.0):
    """Time the FP64 oracle on one configuration (C1 static drop 128^2,
    2 lattices; C3 coupled drop 1024x512) with the OpenMP threads this process
    was started with: at least two steps and about min_s seconds."""
    import oracle
    from paper_2504_09024_amd import workloads as W
    p, fl = W.static_drop() if name == "c1" else W.shear_drop()
    o = oracle.OracleSim(oracle.make_params(**p), fl["phi"], fl["c"], fl.get("ux"), fl.get("uy"))
    steps, dt = 0, 0.0
    while steps < 2 or dt < min_s:
        t0 = time.perf_counter()
        o.run(1 if steps < 2 else max(1, steps))
        dt += time.perf_counter() - t0
        steps += 1 if steps < 2 else max(1, steps)
    return {"config": name, "threads": oracle.num_threads(), "steps": steps,
            "MLUPS": round(p["nx"] * p["ny"] * steps / dt / 1e6, 3)}


def oracle_timing():
    """The oracle on C1 and C3, single-threaded and on every core this
    process may use; one JSON line with the host's CPU model."""
    import subprocess
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next(ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name"))
    except (OSError, StopIteration):
        pass
    legs = []
    for name in ("c1", "c3"):
        for threads in (1, cores):
            env = dict(os.environ, OMP_NUM_THREADS=str(threads))
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-leg", name],
                               env=env, capture_output=True, text=True, check=True)
            legs.append(json.loads(r.stdout.strip().splitlines()[-1]))
            log(f"[bench] oracle {legs[-1]}")
    print(json.dumps({"oracle_timing": legs, "cpu_model": model, "cores": cores}), flush=True)


WORKLOADS = ("batched", "c3", "c1", "c2", "e1", "e2", "c5", "calib")
# storage forms reported beside the headline: the batch, the single
# 1024x512 drop and the 3D drop
FORM_WORKLOADS = ("batched", "c3", "c5")


def copy_ceiling(torch, cmlb, stream, mib=2048, reps=20, planes=None):
    """Read + write GB/s of the library's plain copy (non-temporal loads and
    stores) with two buffers of `mib` MiB: the practical HBM ceiling on the
    device the benchmark runs on.  With `planes` (9 or 27) the buffers are
    split into that many planes copied side by side (cmlb_copy_planes): the
    same ceiling for a structure-of-arrays access with that many read and
    write streams open at once."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    if planes:
        # whole 4 KiB pages per plane, so that no plane starts inside a
        # cache line (the populations' direction planes do not either)
        plane_bytes = (4 * n // planes) // 4096 * 4096
        moved = 2 * planes * plane_bytes

        def run():
            cmlb.device_copy_planes(a.data_ptr(), b.data_ptr(), plane_bytes, planes, True, stream)
    else:
        moved = 2 * 4 * n

        def run():
            cmlb.device_copy(a.data_ptr(), b.data_ptr(), 4 * n, True, stream)
    for _ in range(3):
        run()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        run()
    e1.record()
    torch.cuda.synchronize()
    gbps = moved * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    return gbps


def workload(W, name):
    if name == "batched":
        sims = W.batched_shear_drops(64)
        desc = ("64 seeded coupled surfactant-laden shear drops (default_rng(2504)): sizes "
                "256x256..1024x512, R=ny/8, Ca~U[0.05,0.6], E~U[0.1,0.5], c0~U[0.1,0.5], "
                "Pe_s log-U[0.5,10], Re=0.1, Pe*=0.5, walls at +-U0; one launch per step")
    elif name == "c3":
        sims = [W.shear_drop()]
        desc = ("coupled surfactant-laden shear drop, 1024x512, R=64, Ca=0.3, E=0.2, "
                "c0/c_max=0.3, Re=0.1, walls at +-U0")
    elif name == "c1":
        sims = [W.static_drop()]
        desc = "static drop, 128x128 periodic, R=32, W=4, D_s=0.01, phi and c lattices"
    elif name == "c2":
        sims = [W.vortex_drop()]
        desc = ("drop in a time-reversing single vortex, 512x512 periodic, R=64, U0=0.02, "
                "T=20000, phi and c lattices")
    elif name == "e1":
        sims = [W.static_drop(n=512, R=128.0, D_s=d) for d in (0.05, 0.1, 0.2)]
        desc = ("three static drops (Sec. 4.1), 512x512 periodic, R=128, W=4, "
                "D_s in {0.05, 0.1, 0.2}, phi and c lattices, one launch per step")
    elif name == "c5":
        sims = [W.shear_drop3()]
        desc = ("3D (D3Q27) coupled surfactant-laden drop in shear, 256x128x128, R=32, Ca=0.3, "
                "E=0.2, c0/c_max=0.3, Re=0.1, walls at +-U0; moments and collision launches")
    elif name == "calib":
        sims = [W.shear_drop(nx=4096, ny=2048)]
        desc = ("roofline calibration: one coupled surfactant-laden shear drop, 4096x2048, "
                "R=256, Ca=0.3, E=0.2, c0/c_max=0.3, Re=0.1, walls at +-U0 (0.9 GB per FP32 "
                "copy of the populations)")
    elif name == "e2":
        sims = [W.advected_drop()]
        desc = ("drop in a uniform flow (Sec. 4.2), 1024x512 periodic, R=128, D_s=0.1, "
                "U0=512/T_D, phi and c lattices")
    else:
        raise ValueError(name)
    return sims, desc


def lattices_of(sims):
    return 3 if sims[0][0].get("flow") == "coupled" else 2


def q_of(sims):
    return 27 if "nz" in sims[0][0] else 9


def nodes_of(sims):
    return sum(p["nx"] * p["ny"] * p.get("nz", 1) for p, _ in sims)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16"])
    ap.add_argument("--workload", default="batched", choices=list(WORKLOADS))
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--tile-width", type=int, default=0, help="64 or 128 (with --tile-rows)")
    ap.add_argument("--tile3", default="", help="3D collision column ty,zs (e.g. 4,16)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-xcd-remap", action="store_true")
    ap.add_argument("--stores", default="auto", choices=["auto", "default", "nt"],
                    help="cache policy of the population stores (default: library's choice)")
    ap.add_argument("--tile-group", type=int, default=-1,
                    help="column-group width of the tile order (default: library's)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shape instead of timing the options")
    ap.add_argument("--no-forms", action="store_true", help="skip the other storage forms")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--launch-costs", action="store_true",
                    help="print the cost of a grid barrier and of a graph kernel boundary")
    ap.add_argument("--copy-bw", default="", metavar="MIB,MIB,...",
                    help="only time torch device copies of these sizes (GB/s read + write)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (the reference "
                         "kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--record-traffic", nargs=4, default=None,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="(no GPU) turn rocprofv3 counter_collection.csv files of the step "
                         "kernel (--workload/--precision) and of the copy calibration into "
                         "profiles/traffic.json")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="(no GPU) time the FP64 CPU oracle on C1 and C3, 1 thread and all cores")
    ap.add_argument("--oracle-leg", default="", help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.oracle_leg:
        print(json.dumps(oracle_leg(args.oracle_leg)), flush=True)
        return
    if args.oracle_timing:
        oracle_timing()
        return

    if args.record_traffic:
        from paper_2504_09024_amd import workloads as W
        sims, _ = workload(W, args.workload)
        dim3 = "nz" in sims[0][0]
        ent = record_traffic(f"{args.workload}:{args.precision}", nodes_of(sims), args.precision,
                             *args.record_traffic,
                             copy_bytes=(args.copy_calibration or 1024) << 20,
                             lattices=lattices_of(sims), q=q_of(sims),
                             kernels=("k_moments3", "k_collide3") if dim3 else ("k_step",))
        print(json.dumps(ent))
        return

    if args.gpus != 1:
        print(f"bench.py: the library steps its simulations on one GPU only (got --gpus "
              f"{args.gpus}); sharding over several GPUs is not implemented", file=sys.stderr)
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

    if args.launch_costs:
        # what separates time steps costs: a grid barrier inside one
        # cooperative launch against a kernel boundary inside a replayed graph
        out = {}
        for blocks in (32, 64, 128, 256):
            sync_us, node_us = cmlb.launch_costs(blocks, 2048)
            out[str(blocks)] = {"grid_sync_us": round(sync_us, 3), "graph_node_us": round(node_us, 3)}
        print(json.dumps({"launch_costs_by_workgroups": out}), flush=True)
        return

    if args.copy_bw:
        # device-to-device copy bandwidth (read + write bytes) at working
        # sets matching the workloads: context for their roofline fractions
        out = {}
        for mib in [int(v) for v in args.copy_bw.split(",")]:
            n = mib * (1 << 20) // 4
            a = torch.ones(n, dtype=torch.float32, device="cuda")
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = max(5, min(200, (8 << 30) // (2 * 4 * n)))
            e0.record()
            for _ in range(reps):
                b.copy_(a)
            e1.record()
            torch.cuda.synchronize()
            out[f"{mib}MiB"] = round(2 * 4 * n * reps / (e0.elapsed_time(e1) / 1e3) / 1e9, 1)
            # the library's own copy kernel, default and non-temporal loads
            # and stores
            for nt in (False, True):
                for _ in range(3):
                    cmlb.device_copy(a.data_ptr(), b.data_ptr(), 4 * n, nt, stream)
                e0.record()
                for _ in range(reps):
                    cmlb.device_copy(a.data_ptr(), b.data_ptr(), 4 * n, nt, stream)
                e1.record()
                torch.cuda.synchronize()
                key = f"{mib}MiB_lib_{'nt' if nt else 'default'}"
                out[key] = round(2 * 4 * n * reps / (e0.elapsed_time(e1) / 1e3) / 1e9, 1)
            del a, b
            # the same bytes as 9 and 27 planes copied side by side
            for planes in (9, 27):
                out[f"{mib}MiB_lib_nt_{planes}planes"] = round(
                    copy_ceiling(torch, cmlb, stream, mib=mib, reps=reps, planes=planes), 1)
        print(json.dumps({"copy_GBps_read_plus_write": out}), flush=True)
        return

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4,
                          "launches": 5}))
        return

    sims, desc = workload(W, args.workload)
    dim3 = "nz" in sims[0][0]
    nodes = nodes_of(sims)
    prec = args.precision
    log(f"[bench] workload {args.workload} ({len(sims)} sims, {nodes} nodes), {prec}, "
        f"warmup {args.warmup}, steps {args.steps}")
    if dim3:
        ctx = make_ctx3(cmlb, sims, prec, stream, not args.no_graph,
                        tuple(int(v) for v in args.tile3.split(",")) if args.tile3 else None,
                        args.stores)
    else:
        ctx = make_ctx(cmlb, sims, prec, stream, args.tile_rows, not args.no_graph,
                       not args.no_xcd_remap, args.tile_group, args.stores, args.tile_width)
    tuned = None
    if dim3 and not args.no_autotune and not args.tile3 and args.stores == "auto":
        tuned = ctx.autotune(20)
        log(f"[bench] autotuned launch: 64x{tuned[0]} columns over {tuned[1]} planes, "
            f"{tuned[2]} stores")
        tuned = (f"64x{tuned[0]} columns over {tuned[1]} planes", None, tuned[2])
    elif not dim3 and not args.no_autotune and not args.tile_rows and args.stores == "auto":
        tuned = ctx.autotune(20)
        log(f"[bench] autotuned launch: {tuned[0]}x{tuned[1]} tiles, {tuned[2]} stores")
    gpu_s, wall_s = timed_run(ctx, args.steps, args.warmup, torch)
    inv = ctx.inventory(0)
    ctx.close()
    mlups = nodes * args.steps / gpu_s / 1e6
    ms_per_step = gpu_s * 1e3 / args.steps
    lat = lattices_of(sims)
    bpl = algorithmic_bytes_per_node(prec, lat, q_of(sims)) * nodes
    achieved = bpl / (gpu_s / args.steps) / 1e9
    log(f"[bench] {mlups:.0f} MLUPS, {ms_per_step * 1e3:.2f} us/step, {achieved:.0f} GB/s "
        f"({achieved / HBM_PEAK_GBS:.3f} of peak; wall {wall_s:.3f} s)")

    # the plain-copy ceiling on this device, measured in the same run
    copy_gbps = copy_ceiling(torch, cmlb, stream)
    copy27_gbps = copy_ceiling(torch, cmlb, stream, planes=27)
    traffic = traffic_entry(args.workload, prec, 3 if dim3 else 2)
    log(f"[bench] copy ceiling {copy_gbps:.0f} GB/s (27 planes side by side: "
        f"{copy27_gbps:.0f} GB/s): step at {achieved / copy_gbps:.3f} of it in algorithmic bytes")

    forms = {f"{args.workload}_{prec}": {"MLUPS": round(mlups, 1),
                                         "hbm_frac": round(achieved / HBM_PEAK_GBS, 4)}}
    if not args.no_forms:
        for wl in FORM_WORKLOADS:
            wsims, _ = workload(W, wl) if wl != args.workload else (sims, None)
            wnodes = nodes_of(wsims)
            for fp in ("fp64", "fp32", "fp16"):
                key = f"{wl}_{fp}"
                if key in forms:
                    continue
                if "nz" in wsims[0][0]:
                    c2 = make_ctx3(cmlb, wsims, fp, stream)
                else:
                    c2 = make_ctx(cmlb, wsims, fp, stream)
                k = {"batched": 200, "c3": 2000, "c5": 200}[wl]
                s, _ = timed_run(c2, k, 20, torch)
                c2.close()
                bw = (algorithmic_bytes_per_node(fp, lattices_of(wsims), q_of(wsims)) * wnodes
                      / (s / k) / 1e9)
                forms[key] = {"MLUPS": round(wnodes * k / s / 1e6, 1),
                              "hbm_frac": round(bw / HBM_PEAK_GBS, 4)}
                log(f"[bench] form {key}: {forms[key]}")
        for wl in FORM_WORKLOADS:
            base = forms.get(f"{wl}_fp64", {}).get("MLUPS")
            for fp in ("fp64", "fp32", "fp16"):
                key = f"{wl}_{fp}"
                if base and key in forms:
                    forms[key]["speedup_vs_fp64_gpu"] = round(forms[key]["MLUPS"] / base, 2)

    cpu = None
    if not args.no_cpu:
        log("[bench] CPU oracle sample")
        cpu = cpu_baseline(sims)
        log(f"[bench] CPU oracle: {cpu}")

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
            "workload": desc,
            "sims": len(sims), "nodes": nodes, "storage": prec, "lattices": lat,
            "velocities": q_of(sims),
            "graph": not args.no_graph, "tile_rows": args.tile_rows or "default",
            "tile_width": args.tile_width or "default",
            "xcd_remap": not args.no_xcd_remap,
            "tile_group": args.tile_group if args.tile_group >= 0 else "default",
            "stores": args.stores,
            "autotuned": ((f"{tuned[0]}, {tuned[2]} stores" if tuned[1] is None else
                           f"{tuned[0]}x{tuned[1]} tiles, {tuned[2]} stores") if tuned else None),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
        },
        "copy_ceiling": {
            "value": round(copy_gbps, 1), "unit": "GB/s",
            "kernel": "cmlb_copy, non-temporal loads and stores, two 2 GiB buffers",
            "achieved_over_copy": round(achieved / copy_gbps, 4),
            "traffic_over_copy": (round(traffic / (ms_per_step / 1e3) / 1e9 / copy_gbps, 4)
                                  if traffic else None),
            # the 2D coupled step reads and writes 27 direction planes
            # (3 lattices x 9) at once
            "planes27": {
                "value": round(copy27_gbps, 1),
                "kernel": "cmlb_copy_planes, 27 planes, non-temporal, two 2 GiB buffers",
                "achieved_over": round(achieved / copy27_gbps, 4),
                "traffic_over": (round(traffic / (ms_per_step / 1e3) / 1e9 / copy27_gbps, 4)
                                 if traffic else None),
            },
        },
        "cpu_baseline": cpu,
        "forms": forms,
        "inventory_sim0": {"phi": inv[0], "c": inv[1]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
