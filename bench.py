"""Throughput of the fused phase-field power-law D2Q9 step on one MI355X.

Default workload: one 2048 x 4096 domain with 64 seeded bubbles in a
shear-thinning power-law liquid (n = 0.6), density ratio 1000, float32
arithmetic.  A "step" is one time step of the whole domain (collision,
streaming, bounce-back, phase-field update); the timed region covers exactly
`--steps` steps with the state resident in HBM.  The tile variant is chosen by
the autotuner before timing.  Prints one JSON line; the "forms" object adds
the batched 48-case sweep (batched vs one by one), the stored-hbar form,
the float16 storage form, the three-component system on the same domain and
the smaller configurations.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the step kernel on the default 2048 x 4096 workload,
# from rocprofv3 FETCH_SIZE and WRITE_SIZE runs scaled by the same counters
# read for a 512 MiB device copy (x 1.9999 and x 1.0).  Valid only for the kernel
# sources they were taken on (sha256 prefix of pflbm_step.hip + pflbm_device.h)
# and the same tile variant; otherwise the bench reports null.
MEASURED_TRAFFIC = {"source_sha256": "4f41d287dbabd5e7", "variant": "tile32x16_t512",
                    "nx": 2048, "ny": 4096, "bytes_per_launch": 899.1e6}

# VALU instructions per lattice update of the same kernel (rocprofv3
# SQ_INSTS_VALU / SQ_WAVES: one wave per 64 updates, halo work included),
# under the same conditions as MEASURED_TRAFFIC.  The VALU issue ceiling of
# MI355X without packed float32: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz =
# 39.3 T lane-instructions/s.
MEASURED_VALU = {"source_sha256": "4f41d287dbabd5e7", "variant": "tile32x16_t512",
                 "nx": 2048, "ny": 4096, "instr_per_update": 1002.1}
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9

# steps per captured hipGraph in the graph-replay forms
GRAPH_STEPS = 50


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nx", type=int, default=2048)
    ap.add_argument("--ny", type=int, default=4096)
    ap.add_argument("--bubbles", type=int, default=64)
    ap.add_argument("--variant", type=int, default=-1, help="tile variant; -1 autotunes")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched and stored-hbar forms")
    ap.add_argument("--storage", type=int, default=0, choices=(0, 1),
                    help="state form of the timed workload: 0 float32 deviations, 1 float16 pair moments")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (calibrates HBM byte counters)")
    return ap.parse_args()


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("pflbm_step.hip", "pflbm_device.h"):
        with open(os.path.join(ROOT, "paper_2207_09431_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_for(m, key, variant, nx, ny, storage=0):
    """A stored profiler figure if it was taken on these kernel sources,
    this variant and domain (float32 form), else None."""
    if storage != 0:
        return None
    try:
        same = kernel_source_hash() == m["source_sha256"]
    except OSError:
        same = False
    if same and variant == m["variant"] and (nx, ny) == (m["nx"], m["ny"]):
        return m[key]
    return None


def measured_traffic(variant, nx, ny, storage=0):
    return measured_for(MEASURED_TRAFFIC, "bytes_per_launch", variant, nx, ny, storage)


def copy_bandwidth(torch, mib=1024, reps=10):
    """GB/s (bytes read + written) of a plain device-to-device copy of `mib`
    MiB on this GPU: the attainable side of the HBM roofline."""
    n = mib << 20
    x = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * n / (ms * 1e-3) / 1e9


def timed_steps(torch, solvers, steps, warmup):
    """Milliseconds per step for advancing every solver by one step per step
    (all on the current stream), measured with events on that stream."""
    for s in solvers:
        s.step(warmup)
    torch.cuda.synchronize()
    stream = solvers[0].stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for s in solvers:
        s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, time.perf_counter() - t0


def cpu_baseline(case, seconds):
    """The FP64 oracle on the same workload as the timed GPU run (the full
    domain, same seeded fields), for about `seconds` of wall time, its per-node
    loops split over every core OpenMP is given (OMP_NUM_THREADS where the
    host sets it, else the cores this process may run on); the steps timed are
    as many as fit in that time, and the rate is extrapolated from them.  One
    more step runs on a single thread."""
    from oracle.pfo import Oracle, set_threads, get_threads
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    threads_wanted = int(env) if env.isdigit() and int(env) > 0 else cores
    set_threads(threads_wanted)
    threads = get_threads()
    o = Oracle(case["params"])
    o.init_fields(case["C"], case["u"], case["p"])
    cells = case["params"]["nx"] * case["params"]["ny"]
    t = time.perf_counter()
    o.step(1)
    per = time.perf_counter() - t
    n = max(2, int(seconds / max(per, 1e-6)))
    t = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t
    set_threads(1)
    t = time.perf_counter()
    o.step(1)
    dt1 = time.perf_counter() - t
    set_threads(threads_wanted)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(cells * n / dt / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{case['name']}, the full {case['params']['nx']}x{case['params']['ny']} domain of the timed "
                      f"workload: {n} steps after one warm-up step ({dt:.1f} s), float64, {threads} OpenMP threads "
                      f"({cores} cores visible to the process)",
            "single_thread_value": round(cells / dt1 / 1e6, 3), "single_thread_steps": 1,
            "cpu_model": model}


def small_configs(torch, Solver, inputs, steps, warmup):
    """The smaller configurations (cache-resident, bound by the latency of one
    tile's step): the 64 x 128 rising bubble, a 200 x 400 power-law bubble
    (d = 40) and the 256 x 512 three-component case; plain launches and
    hipGraph replay of GRAPH_STEPS steps (timed after two warm-up replays)."""
    out = {}
    for name, case in (("rising_bubble_64x128", inputs.rising_bubble_small()),
                       ("powerlaw_bubble_200x400", inputs.powerlaw_bubble(n=0.8, d=40.0)),
                       ("three_component_256x512", inputs.three_component())):
        s = Solver(case["params"])
        s.init_fields(0, case["C"], case["u"], case["p"])
        var = s.autotune(steps=3)
        cells = case["params"]["nx"] * case["params"]["ny"]
        ms, _ = timed_steps(torch, [s], steps, warmup)
        s.set_graph(GRAPH_STEPS)
        ms_g, _ = timed_steps(torch, [s], max(GRAPH_STEPS, steps - steps % GRAPH_STEPS), 2 * GRAPH_STEPS)
        out[name] = {"mlups": round(cells / (ms * 1e-3) / 1e6, 1), "graph_mlups": round(cells / (ms_g * 1e-3) / 1e6, 1),
                     "ms_per_step": round(ms, 4), "variant": var, "bytes_per_update": s.bytes_per_update()}
        s.close()
    return out


def batch_forms(torch, Solver, inputs, steps, warmup):
    """48 uneven bubble cases (16 each of 150x300, 200x400, 300x600): one
    batched launch per step vs the same cases advanced one by one."""
    cases = inputs.batch_sweep()
    cells = sum(c["params"]["nx"] * c["params"]["ny"] for c in cases)
    b = Solver([c["params"] for c in cases])
    for k, c in enumerate(cases):
        b.init_fields(k, c["C"], c["u"], c["p"])
    bvar = b.autotune(steps=3)
    ms_b, _ = timed_steps(torch, [b], steps, warmup)
    b.set_graph(GRAPH_STEPS)                       # the same launches replayed from a hipGraph
    ms_g, _ = timed_steps(torch, [b], max(GRAPH_STEPS, steps - steps % GRAPH_STEPS), 2 * GRAPH_STEPS)
    b.set_graph(0)
    singles = []
    for c in cases:
        s = Solver(c["params"])
        s.init_fields(0, c["C"], c["u"], c["p"])
        s.set_variant(s.variants().index(bvar))
        singles.append(s)
    ms_s, _ = timed_steps(torch, singles, steps, warmup)
    return {"cases": len(cases), "cells": cells, "variant": bvar,
            "batched_mlups": round(cells / (ms_b * 1e-3) / 1e6, 1),
            "batched_graph_mlups": round(cells / (ms_g * 1e-3) / 1e6, 1),
            "one_by_one_mlups": round(cells / (ms_s * 1e-3) / 1e6, 1),
            "batched_ms_per_step": round(ms_b, 4), "one_by_one_ms_per_step": round(ms_s, 4)}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): every workload here is advanced "
              "by a single device", file=sys.stderr)
        sys.exit(2)
    import torch
    if a.copy_probe > 0:
        n = a.copy_probe * (1 << 20)
        x = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "launches": 5}), flush=True)
        return
    from paper_2207_09431_amd import inputs
    from paper_2207_09431_amd.pflbm import Solver

    case = inputs.many_bubbles(a.nx, a.ny, a.bubbles)
    prm = dict(case["params"], storage=a.storage)
    s = Solver(prm, device="cuda:0")
    s.init_fields(0, case["C"], case["u"], case["p"])
    if a.variant >= 0:
        s.set_variant(a.variant)
        variant = s.variants()[a.variant]
        tuning = None
    else:
        variant = s.autotune(steps=5)
        tuning = {k: round(v, 4) for k, v in s.tuning.items()}
    torch.cuda.synchronize()
    cells = prm["nx"] * prm["ny"]

    ms, wall = timed_steps(torch, [s], a.steps, a.warmup)
    mlups = cells / (ms * 1e-3) / 1e6
    diag = s.bubble_centroid_velocity(0, 0)
    bpu = s.bytes_per_update()
    achieved = bpu * cells / (ms * 1e-3) / 1e9
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
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{case['name']}: {a.nx}x{a.ny} single domain, {a.bubbles} seeded bubbles R 25-40, "
                        f"power-law liquid n=0.6 K=0.1, density ratio 1000, float32 arithmetic with the "
                        f"phase field, the gbar level, their stencils and the bulk chemical potential in float64, "
                        + ("state: gbar level float64 + 8 deviations float32, C float64, tau float32 (tau_h = 1/2)"
                           if a.storage == 0 else
                           "state: gbar level float64 + momentum float32 + 6 float16 pair moments, C float64, "
                           "tau float32 (tau_h = 1/2)"),
            "nx": a.nx, "ny": a.ny, "cells": cells, "bytes_per_update": bpu, "kernel_variant": variant,
            "autotune_ms_per_step": tuning, "wall_s_timed": round(wall, 4), "gas_mass": diag[0],
        },
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(variant, a.nx, a.ny, a.storage)},
    }
    vpu = measured_for(MEASURED_VALU, "instr_per_update", variant, a.nx, a.ny, a.storage)
    if vpu is not None:
        ceiling = VALU_ISSUE_PEAK / vpu / 1e6
        out["roofline"]["valu"] = {"instr_per_update": vpu, "issue_peak_per_s": VALU_ISSUE_PEAK,
                                   "ceiling_mlups": round(ceiling, 1), "frac": round(mlups / ceiling, 4)}
    else:
        out["roofline"]["valu"] = None
    del s
    torch.cuda.empty_cache()
    copy_gbs = copy_bandwidth(torch)
    out["roofline"]["measured_copy_GBs"] = round(copy_gbs, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / copy_gbs, 4)
    if not a.no_forms:
        forms = {"batched_48": batch_forms(torch, Solver, inputs, max(20, a.steps // 4), 5)}
        torch.cuda.empty_cache()
        sh = Solver(dict(prm, store_h=1), device="cuda:0")
        sh.init_fields(0, case["C"], case["u"], case["p"])
        sh.set_variant(sh.variants().index(variant))
        ms_h, _ = timed_steps(torch, [sh], max(20, a.steps // 4), 5)
        forms["stored_hbar"] = {"mlups": round(cells / (ms_h * 1e-3) / 1e6, 1), "ms_per_step": round(ms_h, 4),
                                "bytes_per_update": sh.bytes_per_update(),
                                "achieved_GBs": round(sh.bytes_per_update() * cells / (ms_h * 1e-3) / 1e9, 1)}
        del sh
        torch.cuda.empty_cache()
        sq = Solver(dict(prm, storage=1), device="cuda:0")
        sq.init_fields(0, case["C"], case["u"], case["p"])
        qvar = sq.autotune(steps=5)
        ms_q, _ = timed_steps(torch, [sq], max(20, a.steps // 4), 5)
        forms["float16_storage"] = {"mlups": round(cells / (ms_q * 1e-3) / 1e6, 1), "ms_per_step": round(ms_q, 4),
                                    "variant": qvar, "bytes_per_update": sq.bytes_per_update(),
                                    "achieved_GBs": round(sq.bytes_per_update() * cells / (ms_q * 1e-3) / 1e9, 1)}
        del sq
        torch.cuda.empty_cache()
        # the three-component system (two phase fields) on the same domain
        tc = inputs.three_component(nx=a.nx, ny=a.ny)
        st = Solver(tc["params"], device="cuda:0")
        st.init_fields(0, tc["C"], tc.get("u"), tc.get("p"))
        tvar = st.autotune(steps=5)
        ms_t, _ = timed_steps(torch, [st], max(20, a.steps // 4), 5)
        forms["three_component"] = {"mlups": round(cells / (ms_t * 1e-3) / 1e6, 1), "ms_per_step": round(ms_t, 4),
                                    "variant": tvar, "bytes_per_update": st.bytes_per_update(),
                                    "achieved_GBs": round(st.bytes_per_update() * cells / (ms_t * 1e-3) / 1e9, 1)}
        del st
        torch.cuda.empty_cache()
        forms["small_configs"] = small_configs(torch, Solver, inputs, max(100, a.steps), 20)
        out["forms"] = forms
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
