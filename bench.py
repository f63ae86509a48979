"""Throughput of the fused phase-field power-law D2Q9 step on one MI355X.

Default workload: one 2048 x 4096 domain with 64 seeded bubbles in a
shear-thinning power-law liquid (n = 0.6), density ratio 1000, float32.  A
"step" is one time step of the whole domain (collision, streaming,
bounce-back, phase-field update); the timed region covers exactly `--steps`
steps with the inputs resident in HBM.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nx", type=int, default=2048)
    ap.add_argument("--ny", type=int, default=4096)
    ap.add_argument("--bubbles", type=int, default=64)
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--store-h", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def cpu_baseline(seconds):
    """The FP64 oracle, single-threaded, on the 256 x 512 window case of the
    same seeded workload, for about `seconds` of CPU time."""
    from oracle.pfo import Oracle
    from paper_2207_09431_amd import inputs
    case = inputs.many_bubbles_crop()
    o = Oracle(case["params"])
    o.init_fields(case["C"], case["u"], case["p"])
    cells = case["params"]["nx"] * case["params"]["ny"]
    t = time.perf_counter()
    o.step(2)
    per = (time.perf_counter() - t) / 2
    n = max(3, int(seconds / max(per, 1e-6)))
    t = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t
    return {"value": cells * n / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{case['name']} (256x512 window of the same seed), {n} steps, float64, one thread"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the method's domain is advanced by "
              "one device here", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2207_09431_amd import inputs
    from paper_2207_09431_amd.pflbm import Solver

    case = inputs.many_bubbles(a.nx, a.ny, a.bubbles)
    prm = dict(case["params"])
    prm["store_h"] = a.store_h
    s = Solver(prm, device="cuda:0")
    if a.variant >= 0:
        s.set_variant(a.variant)
    s.init_fields(0, case["C"], case["u"], case["p"])
    torch.cuda.synchronize()
    cells = prm["nx"] * prm["ny"]

    s.step(a.warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    stream = s.stream
    t0 = time.perf_counter()
    ev0.record(stream)
    s.step(a.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / a.steps
    mlups = cells / (ms * 1e-3) / 1e6

    diag = s.bubble_centroid_velocity(0, 0)
    bpu = s.bytes_per_update()
    achieved = bpu * cells / (ms * 1e-3) / 1e9
    variant = s.variants()[s_variant(s, a.variant)]
    out = {
        "metric": "MLUPS (D2Q9 g+h)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{case['name']}: {a.nx}x{a.ny} single domain, {a.bubbles} seeded bubbles R 25-40, "
                        f"power-law liquid n=0.6 K=0.1, density ratio 1000, float32 "
                        f"{'stored hbar' if a.store_h else 'C_i state (tau_h=1/2)'}",
            "nx": a.nx, "ny": a.ny, "cells": cells, "bytes_per_update": bpu, "kernel_variant": variant,
            "wall_s_timed": round(wall, 4), "gas_mass": diag[0],
        },
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    print(json.dumps(out), flush=True)


def s_variant(s, requested):
    return requested if requested >= 0 else 0


if __name__ == "__main__":
    main()
