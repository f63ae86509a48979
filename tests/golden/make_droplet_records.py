"""Writes droplet_constant.json and droplet_vm_link.json: the oracle's bubble
diagnostics (Sec. 3.1; Sec. 4.2 Eqs. (43)-(44)) of both dispersed components
of the Sec. 3.1 three-component system (inputs.bubble_droplet: a light
bubble rising towards a droplet, 200 x 400), every 1,000 steps up to 10,000,
with constant mobility and the default (mixed-difference) hbar forcing, and
with variable mobility (Eq. (6)), the diffusion source in the conservative
link form and central differences in the hbar forcing.  Calls only the
oracle and the seeded input recipe; takes about five minutes per record on
8 threads.

    python tests/golden/make_droplet_records.py [threads]
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.pfo import Oracle, set_threads  # noqa: E402
from paper_2207_09431_amd import inputs  # noqa: E402

EVERY, LAST = 1000, 10000
# record file: (variable_mobility, switches over the recipe's parameters)
RECORDS = {"droplet_constant.json": (0, {"hforce_cd": 0}),
           "droplet_vm_link.json": (1, {"mobility_flux": 1})}


def record(name, vm, over):
    case = inputs.bubble_droplet(variable_mobility=vm, hforce_cd=1 if vm else 0)
    o = Oracle(dict(case["params"], **over))
    o.init_fields(case["C"], case.get("u"), case.get("p"))
    rows = []
    for n in range(EVERY, LAST + 1, EVERY):
        o.step(EVERY)
        row = {"step": n}
        for k in (0, 1):
            mass, above, xc, yc, ux, uy = (float(v) for v in o.centroid(k))
            row[f"c{k + 1}"] = {"mass": mass, "mass_above_half": above, "y_c": yc, "V_y": uy}
        rows.append(row)
        print(name, rows[-1], flush=True)
    out = {"case": case["name"] + ("_link" if vm else ""), "variable_mobility": vm, "switches": over,
           "source": "oracle/pfo.c via tests/golden/make_droplet_records.py", "samples": rows}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), name), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


def main():
    set_threads(int(sys.argv[1]) if len(sys.argv) > 1 else min(16, os.cpu_count() or 1))
    for name, (vm, over) in RECORDS.items():
        record(name, vm, over)


if __name__ == "__main__":
    main()
