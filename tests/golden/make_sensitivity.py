"""Write tests/golden/sensitivity.json: how strongly the long-horizon
workloads themselves amplify a perturbation at FP32 scale, measured with the
FP64 oracle alone (nothing here runs on or reads from the GPU library).

For each workload the oracle runs three times from the same seeded initial
fields (paper_2504_09024_amd.workloads):

  base      the FP64 oracle as it is;
  perturbed phi of the initial fields multiplied by (1 + 2^-24 s) with a
            seeded random sign s per node (one FP32 rounding of phi, once);
  fp32      after every step each stored population is rounded to the
            nearest FP32 value (ties to even) in the storage form of the
            FP32 library, s_a = q_a / w_a - q_ref with q_ref = 0 for f and h
            and rho_b cs^2 for g: FP32 storage rounding alone, with the
            arithmetic left in FP64.

and records the relative L2 differences of phi, c and u (as one vector field)
between base and each of the others at every checkpoint.  The C3 coupled
shear drop (1024x512, Sec. 4.3 set-up, Re = 0.1, Ca in {0.1, 0.3, 0.5},
E = 0.2, c0 = 0.3) is checked at 1000 and 5000 steps, the C2 drop in the
time-reversing vortex (512x512, Sec. 4.2 extended; T = 20000) at T/4, T/2 and
T, the 3D C5 drop in shear scaled down to 64x32x32 (R = 8) at 1000 and 5000
steps, a 256x128 scale-down of C3 at 1000 steps, the C1 static drop (128x128,
Sec. 4.1 set-up) at 500 and 2000 steps and the random-field parity case
coupled_random at 150 steps (the last three cheap enough for the CPU suite
to recompute).

Usage (OpenMP threads from OMP_NUM_THREADS; results do not depend on them):
    python tests/golden/make_sensitivity.py [--only KEY ...] [--cache DIR]
Each run's checkpoint fields are cached under --cache (default
tests/golden/.sensitivity_cache, not committed) so an interrupted generation
resumes; the JSON is rewritten after every finished workload.
"""
from __future__ import annotations

import argparse
import concurrent.futures
import fcntl
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from paper_2504_09024_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "sensitivity.json")
PERTURB = 2.0 ** -24
SEED = 2504


def workloads():
    """key -> (builder, checkpoints), in the order they are generated."""
    from parity_cases import CASES
    out = {"c3_256x128_Ca0.3": (lambda: W.shear_drop(nx=256, ny=128, Ca=0.3), (1000,)),
           "coupled_random": (CASES["coupled_random"][0], (150,)),
           "c1": (lambda: W.static_drop(), (500, 2000))}
    for ca in (0.3, 0.1, 0.5):
        out[f"c3_Ca{ca}"] = (lambda ca=ca: W.shear_drop(Ca=ca), (1000, 5000))
    out["c2"] = (lambda: W.vortex_drop(), (5000, 10000, 20000))
    # 3D: the C5 shear drop scaled down by four in every direction (R = 8)
    out["c5_64x32x32"] = (lambda: W.shear_drop3(nx=64, ny=32, nz=32, R=8.0), (1000, 5000))
    return out


def perturbed_phi(phi):
    s = np.random.default_rng(SEED).choice([-1.0, 1.0], size=phi.shape)
    return phi * (1.0 + PERTURB * s)


def _round_plane(q, w, ref):
    s = q / w
    if ref:
        s -= ref
    s[...] = s.astype(np.float32)
    if ref:
        s += ref
    np.multiply(s, w, out=q)


def round_storage_fp32(o, P_ref, pool):
    """Round the oracle's populations in place to the FP32 storage form, one
    direction plane per task (D2Q9 or D3Q27)."""
    w = oracle.weights3() if o.f.shape[0] == 27 else oracle.weights()
    jobs = [(q[a], w[a], ref) for q, ref in ((o.f, 0.0), (o.h, 0.0), (o.g, P_ref))
            if q is not None for a in range(len(w))]
    list(pool.map(lambda j: _round_plane(*j), jobs))


def make_sim(p, fl, phi):
    if "nz" in p:
        return oracle.OracleSim3(oracle.make_params3(**p), phi, fl["c"], fl.get("ux"),
                                 fl.get("uy"), fl.get("uz"), fl.get("P"))
    return oracle.OracleSim(oracle.make_params(**p), phi, fl["c"], fl.get("ux"), fl.get("uy"),
                            fl.get("P"))


FIELDS = ("phi", "c", "ux", "uy", "uz")


def run_variant(p, fl, variant, checkpoints, label=""):
    phi = perturbed_phi(fl["phi"]) if variant == "perturbed" else fl["phi"]
    o = make_sim(p, fl, phi)
    P_ref = p["rho_b"] / 3.0
    pool = concurrent.futures.ThreadPoolExecutor(max(1, oracle.num_threads()))
    out = {}
    for t_end in checkpoints:
        while o.t < t_end:
            if variant == "fp32":
                fault = o.run(1)
                round_storage_fp32(o, P_ref, pool)
            else:
                fault = o.run(min(250, t_end - o.t))
            if fault:
                raise RuntimeError(f"oracle fault {fault} at t={o.t}")
            if o.t % 1000 == 0:
                print(f"[sensitivity] {label} {variant} t={o.t}", flush=True)
        fl_t = o.fields()
        out[t_end] = {k: fl_t[k].copy() for k in FIELDS if k in fl_t}
    return out


def rel(a, b):
    """Relative L2 difference; None where the base field is zero (u of a
    drop without flow)."""
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0.0 else None


def diffs(base, other):
    uk = [k for k in ("ux", "uy", "uz") if k in base]
    return {"phi": rel(other["phi"], base["phi"]), "c": rel(other["c"], base["c"]),
            "u": rel(np.stack([other[k] for k in uk]), np.stack([base[k] for k in uk]))}


def cached_run(cache, key, p, fl, variant, checkpoints):
    path = os.path.join(cache, f"{key}_{variant}.npz")
    if os.path.exists(path):
        z = np.load(path)
        return {t: {k: z[f"{t}_{k}"] for k in FIELDS if f"{t}_{k}" in z} for t in checkpoints}
    t0 = time.perf_counter()
    res = run_variant(p, fl, variant, checkpoints, key)
    np.savez(path, **{f"{t}_{k}": v for t, d in res.items() for k, v in d.items()})
    print(f"[sensitivity] {key} {variant}: {time.perf_counter() - t0:.0f} s", flush=True)
    return res


def sensitivity(key, builder, checkpoints, cache):
    p, fl = builder()
    runs = {v: cached_run(cache, key, p, fl, v, checkpoints)
            for v in ("base", "perturbed", "fp32")}
    return {str(t): {v: diffs(runs["base"][t], runs[v][t]) for v in ("perturbed", "fp32")}
            for t in checkpoints}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--cache", default=os.path.join(HERE, ".sensitivity_cache"))
    ap.add_argument("--out", default=OUT, help="JSON file the entries are merged into")
    args = ap.parse_args()
    out = args.out
    os.makedirs(args.cache, exist_ok=True)
    note = ("Relative L2 difference of phi, c and u between the FP64 oracle and the "
                     "same oracle run (perturbed) from phi * (1 + 2^-24 s), s a seeded random "
                     "sign per node, or (fp32) with every stored population rounded to FP32 in "
                     "the library's FP32 storage form after each step; written by "
                     "tests/golden/make_sensitivity.py from the oracle alone.")
    for key, (builder, checkpoints) in workloads().items():
        if args.only and key not in args.only:
            continue
        entry = sensitivity(key, builder, checkpoints, args.cache)
        # several generators may run side by side: merge under a lock
        with open(out + ".lock", "w") as lk:
            fcntl.flock(lk, fcntl.LOCK_EX)
            data = {}
            if os.path.exists(out):
                with open(out) as fh:
                    data = json.load(fh)
            data["_note"] = note
            data[key] = entry
            with open(out + ".tmp", "w") as fh:
                json.dump(data, fh, indent=1, sort_keys=True)
                fh.write("\n")
            os.replace(out + ".tmp", out)
        print(f"[sensitivity] {key}: {json.dumps(entry)}", flush=True)


if __name__ == "__main__":
    main()
