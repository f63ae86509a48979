"""Terminal velocities of a set of rising bubbles (Sec. 4.3), advanced
together in one batched solver on the GPU, with the drag post-processing of
Sec. 4.1.

    python -m paper_2207_09431_amd.sweep [--ratio 200] [--cases 3,4,5,6] [--steps 60000] [--scale 2]
        [--mobility constant|variable] [--source product|link] [--hbar-forcing mixed|central]

prints one JSON object per case.  The terminal velocity is read as the
largest sampled mean rise velocity (Eq. (44)) before the bubble comes within
one diameter of the top wall: with constant mobility the gas slowly dissolves
after the plateau, so the velocity peaks on it and then drifts down.
"""
from __future__ import annotations

import argparse
import json

from . import drag, inputs
from .pflbm import PflbmError, Solver


def run_sweep(cases: list, max_steps: int, every: int = 1000, solver_factory=Solver) -> list:
    """Advances all `cases` (single-bubble cases, component 0 the gas) in one
    batched solver for up to `max_steps` steps, sampling the bubble
    diagnostics every `every` steps, and returns per case the samples and the
    report at the terminal sample (None when the case became non-finite or
    never peaked), and why sampling ended ("max_steps", "top_wall" or
    "nonfinite by step N").  `solver_factory` builds the batched solver
    from the list of parameter blocks (the GPU Solver)."""
    s = solver_factory([c["params"] for c in cases])
    for i, c in enumerate(cases):
        s.init_fields(i, c["C"], c.get("u"), c.get("p"))
    samples = [[] for _ in cases]
    alive = [True] * len(cases)
    end = ["max_steps"] * len(cases)
    done = 0
    while done < max_steps and any(alive):
        s.step(every)
        done += every
        for i, c in enumerate(cases):
            if not alive[i]:
                continue
            try:
                diag = s.bubble_centroid_velocity(i, 0)
            except PflbmError as e:
                if e.status != -4:         # only a diverged state ends a case quietly
                    raise
                alive[i] = False
                end[i] = f"nonfinite by step {done}"
                continue
            d = drag.equivalent_diameter(diag[0])
            if diag[3] + 1.5 * d > c["params"]["ny"]:
                alive[i] = False            # within a diameter of the top wall
                end[i] = "top_wall"
                continue
            samples[i].append((done, [float(v) for v in diag]))
    out = []
    for i, c in enumerate(cases):
        res = {"case": c["name"], "steps": samples[i][-1][0] if samples[i] else 0, "end": end[i],
               "samples": samples[i], "report": None}
        if samples[i]:
            # the largest sampled rise velocity, also for a case that ended non-finite
            j = max(range(len(samples[i])), key=lambda q: samples[i][q][1][5])
            res["max_vy"], res["max_vy_step"] = samples[i][j][1][5], samples[i][j][0]
        if samples[i] and not end[i].startswith("nonfinite"):
            k = max(range(len(samples[i])), key=lambda j: samples[i][j][1][5])
            if 0 < k < len(samples[i]) - 1:
                step, diag = samples[i][k]
                res["peak_step"] = step
                res["plateau_change"] = max(abs(samples[i][k + j][1][5] / diag[5] - 1) for j in (-1, 1))
                res["diag"] = diag
        out.append(res)
    # the shape at each case's peak: a second, bitwise identical run of the
    # batch stops at the peak steps in increasing order and copies the gas
    # fraction of the case that peaked there
    order = sorted((r["peak_step"], i) for i, r in enumerate(out) if "peak_step" in r)
    if order:
        s2 = solver_factory([c["params"] for c in cases])
        for i, c in enumerate(cases):
            s2.init_fields(i, c["C"], c.get("u"), c.get("p"))
        at = 0
        for step, i in order:
            if step > at:
                s2.step(step - at)
                at = step
            prm = cases[i]["params"]
            phi = s2.macroscopic(i)["phi"][0].cpu().numpy()
            out[i]["report"] = drag.bubble_report(out[i]["diag"], phi, prm["rho"][2], prm["rho"][0], prm["g"],
                                                  prm["sigma13"], prm["K"], prm["n"])
    return out


def table5_cases(ratio: float, scale: int = 1, mobility: str = "constant", source: str = "product",
                 hbar_forcing: str = "mixed") -> list:
    """The six bubbles of Table 5 at the given density ratio and lattice
    scale, with the mobility (constant or variable, Eq. (6)), the form of the
    diffusion source (product or conservative link form, Eq. (21)) and the
    stencil of the hbar forcing (mixed or central differences) set in every
    case's parameter block."""
    cases = inputs.shear_thinning_sweep(density_ratio=ratio, scale=scale)
    over = dict(variable_mobility=int(mobility == "variable"), mobility_flux=int(source == "link"),
                hforce_cd=int(hbar_forcing == "central"))
    for c in cases:
        c["params"] = dict(c["params"], **over)
    return cases


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--ratio", type=float, default=200.0, help="liquid/gas density ratio (the paper's is 800)")
    ap.add_argument("--cases", default="1,2,3,4,5,6", help="Table 5 cases to run (1-based)")
    ap.add_argument("--steps", type=int, default=None,
                    help="steps on the 200 x 400 lattice (default 60,000); multiplied by scale^2")
    ap.add_argument("--every", type=int, default=None,
                    help="sampling interval on the 200 x 400 lattice (default 1,000); multiplied by scale^2")
    ap.add_argument("--scale", type=int, default=1,
                    help="lattice f times finer than 200 x 400 at the same Re, Eo and Mo")
    ap.add_argument("--mobility", choices=("constant", "variable"), default="constant",
                    help="D_i constant or proportional to C_i (1 - C_i) (Eq. (6))")
    ap.add_argument("--source", choices=("product", "link"), default="product",
                    help="diffusion source of Eq. (21) in the product or the conservative link form")
    ap.add_argument("--hbar-forcing", choices=("mixed", "central"), default="mixed",
                    help="stencil of (e_a - u).grad C_i in the hbar forcing (variable mobility needs central)")
    a = ap.parse_args(argv)
    # at fixed Re, Eo and Mo lattice velocities scale by 1/f and lengths by f,
    # so the same physical time takes f^2 times the steps
    f2 = a.scale * a.scale
    steps = (60000 if a.steps is None else a.steps) * f2
    every = (1000 if a.every is None else a.every) * f2
    all_cases = table5_cases(a.ratio, a.scale, a.mobility, a.source, a.hbar_forcing)
    pick = [int(x) - 1 for x in a.cases.split(",")]
    for r in run_sweep([all_cases[i] for i in pick], steps, every):
        r = dict(r)
        r.pop("samples")
        print(json.dumps(r), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
