"""The stored oracle records in tests/golden come from the oracle as it
stands: the first sample of each shear-thinning record (1,000 steps of a
200 x 400 Table 5 case) is recomputed here and must agree to rounding.
(The other record's first sample needs 8,000 steps of a 128 x 512 case,
minutes on the CPU; its script is the same shape.)"""
import json
import os

import pytest

from oracle.pfo import Oracle
from paper_2207_09431_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("record, ratio, index, suffix, over", [
    ("sweep_case4_terminal.json", 200.0, 3, "", {}),
    ("sweep_case1_cd_terminal.json", 200.0, 0, "_hforce_cd", {"hforce_cd": 1}),
    ("sweep_case4_vm_link.json", 100.0, 3, "_variable_link",
     {"variable_mobility": 1, "mobility_flux": 1, "hforce_cd": 1})])
def test_sweep_record_first_sample_recomputes(record, ratio, index, suffix, over):
    with open(os.path.join(GOLDEN, record)) as f:
        rec = json.load(f)
    first = rec["samples"][0]
    case = inputs.shear_thinning_sweep(density_ratio=ratio)[index]
    assert rec["case"] == case["name"] + suffix
    assert rec.get("switches", over) == over
    o = Oracle(dict(case["params"], **over))
    o.init_fields(case["C"], case["u"], case["p"])
    o.step(first["step"])
    mass, _, _, yc, _, uy = o.centroid(0)
    assert uy == pytest.approx(first["V_y"], rel=1e-9)
    assert yc == pytest.approx(first["y_c"], rel=1e-12)
    assert mass == pytest.approx(first["mass"], rel=1e-12)
