"""GPU runs of the two-layer flow of Sec. 3.3 (Fig. 6) on the paper's 5 x 200
lattice, advanced to steady state and compared with the layered closed form
(Eq. (36), tests/layered.py) in the relative L2 norm of Eq. (35), the
paper's Table 3 errors as bounds (tests/golden); and
GPU-oracle parity on the same setup.

Setup (the paper leaves it open): outer Newtonian layer nu1 = 1/6, inner
consistency K3 = lambda nu1 (lambda^P = K3 / mu1 with rho = 1), truncation
[1e-3, 1], sigma_13 = 5e-4, xi = 4, and the body force chosen so that the
closed-form centre velocity is 0.005, inside the paper's 1e-2 limit.
"""
import json
import os

import numpy as np
import pytest

from oracle.pfo import Oracle
from paper_2207_09431_amd import inputs
from helpers import rel_l2
from layered import force_for_peak, two_layer_profile

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table3_layered_erel.json")
NU1, NU_MIN, NU_MAX, UMAX, NY = 1.0 / 6.0, 1e-3, 1.0, 0.005, 200


@pytest.fixture(scope="module")
def Solver():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_2207_09431_amd.pflbm import Solver as S
    return S


def layered_case(n3, lam):
    G = force_for_peak(UMAX, NY, lam * NU1, n3, NU1, NU_MIN, NU_MAX)
    case = inputs.layered_flow(n3, lam, ny=NY, nu1=NU1, fx=G, nu_min=NU_MIN, nu_max=NU_MAX)
    return case, G


@pytest.mark.parametrize("k", range(8))
def test_layered_flow_within_table3(Solver, k):
    """Steady state: the change of u_x over 2,000 steps below 1e-6 of u_x (the
    float32 state resolves no finer), at most 1.5 million steps."""
    g = json.load(open(GOLDEN))
    n3, lam, bound = g["n3"][k], g["lam"][k], g["E_rel"][k]
    case, G = layered_case(n3, lam)
    s = Solver(case["params"])
    s.init_fields(0, case["C"])
    s.set_graph(100)
    u_old, steps = None, 0
    for _ in range(750):
        s.step(2000)
        steps += 2000
        u = s.macroscopic(0)["u"][0, :, 2].double().cpu().numpy()
        if u_old is not None and np.linalg.norm(u - u_old) < 1e-6 * np.linalg.norm(u):
            break
        u_old = u
    ref = two_layer_profile(NY, G, lam * NU1, n3, NU1, NU_MIN, NU_MAX)
    err = rel_l2(u, ref)
    print(f"n3 {n3} lambda {lam}: {steps} steps, E_rel {err:.4f} (Table 3: {bound}), "
          f"u_max {u.max():.5f} vs {ref.max():.5f}", flush=True)
    s.close()
    assert np.isfinite(u).all() and err <= bound


@pytest.mark.parametrize("k", [0, 7])
def test_layered_flow_parity(Solver, k):
    g = json.load(open(GOLDEN))
    case, _ = layered_case(g["n3"][k], g["lam"][k])
    s = Solver(case["params"])
    s.init_fields(0, case["C"])
    s.step(3000)
    m = {f: v.double().cpu().numpy() for f, v in s.macroscopic(0).items()}
    o = Oracle(case["params"])
    o.init_fields(case["C"])
    o.step(3000)
    om = o.macroscopic()
    ru, rc = rel_l2(m["u"], om["u"]), rel_l2(m["phi"], om["phi"])
    print(f"layered case {k}: rel-L2 u {ru:.2e} C {rc:.2e}", flush=True)
    assert ru <= 1e-5 and rc <= 1e-5
