"""Writes sweep_case4_vm_link.json: the oracle's mean rise velocity,
centroid and component totals of Table 5's case 4 bubble (n = 0.6; 200 x
400, d = 50) at density ratio 100 with variable mobility (Eq. (6)), the
diffusion source in the conservative link form and central differences in
the hbar forcing, every 1,000 steps up to 20,000.  Calls only the oracle and
the seeded input recipe; takes about ten minutes on 8 threads.

    python tests/golden/make_sweep_case4_vm.py [threads]
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.pfo import Oracle, set_threads  # noqa: E402
from paper_2207_09431_amd import inputs  # noqa: E402

EVERY, LAST = 1000, 20000
OVER = {"variable_mobility": 1, "mobility_flux": 1, "hforce_cd": 1}


def main():
    set_threads(int(sys.argv[1]) if len(sys.argv) > 1 else min(16, os.cpu_count() or 1))
    case = inputs.shear_thinning_sweep(density_ratio=100.0)[3]
    o = Oracle(dict(case["params"], **OVER))
    o.init_fields(case["C"], case["u"], case["p"])
    rows = []
    for n in range(EVERY, LAST + 1, EVERY):
        o.step(EVERY)
        mass, above, xc, yc, ux, uy = (float(v) for v in o.centroid(0))
        rows.append({"step": n, "V_y": uy, "y_c": yc, "mass": mass, "mass_above_half": above})
        print(rows[-1], flush=True)
    out = {"case": case["name"] + "_variable_link", "switches": OVER, "source": "oracle/pfo.c via tests/golden/make_sweep_case4_vm.py",
           "samples": rows}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "sweep_case4_vm_link.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
