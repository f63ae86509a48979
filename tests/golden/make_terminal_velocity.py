"""Writes terminal_velocity.json: the oracle's mean rise velocity (Eq. (44))
of the 128 x 512, R = 24, density-ratio-100 bubble at steps 8,000, 9,000 and
10,000, where it sits on its plateau.  Calls only the oracle (and the seeded
input recipe); takes a few minutes on 8 threads.

    python tests/golden/make_terminal_velocity.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.pfo import Oracle, set_threads  # noqa: E402
from paper_2207_09431_amd import inputs  # noqa: E402

STEPS = (8000, 9000, 10000)


def main():
    set_threads(min(16, os.cpu_count() or 1))
    case = inputs.rising_bubble_terminal()
    o = Oracle(case["params"])
    o.init_fields(case["C"], case["u"], case["p"])
    done, rows = 0, []
    for n in STEPS:
        o.step(n - done)
        done = n
        mass, above, xc, yc, ux, uy = o.centroid(0)
        rows.append({"step": n, "V_y": float(uy), "y_c": float(yc), "mass_above_half": float(above)})
        print(rows[-1], flush=True)
    out = {"case": case["name"], "source": "oracle/pfo.c via tests/golden/make_terminal_velocity.py",
           "samples": rows}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "terminal_velocity.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
