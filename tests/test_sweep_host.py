"""Host logic of the sweep driver (terminal-velocity selection, endings,
replay to the peak) with a scripted stand-in for the GPU solver: no GPU and
no oracle involved."""
import math

import numpy as np
import pytest

from paper_2207_09431_amd import sweep
from paper_2207_09431_amd.pflbm import PflbmError

NX, NY, R = 60, 120, 10.0


def disc(yc=40.0):
    y, x = np.mgrid[0:NY, 0:NX].astype(np.float64)
    return 0.5 - 0.5 * np.tanh((np.hypot(x - 30.0, y - yc) - R) / 2.0)


class _Arr:
    def __init__(self, a):
        self.a = a

    def __getitem__(self, i):
        return _Arr(self.a[i])

    def cpu(self):
        return self

    def numpy(self):
        return self.a


class Scripted:
    """Solver stand-in: case i's mean rise velocity follows script[i](step);
    a script returning None makes the case non-finite; y_c rises by the
    velocity's integral."""
    scripts = []

    def __init__(self, params):
        self.n = len(params)
        self.t = 0

    def init_fields(self, i, C, u, p):
        pass

    def step(self, k):
        self.t += k

    def yc(self, i):
        return 40.0 + sum(self.scripts[i](s) or 0.0 for s in range(0, self.t, 100)) * 100

    def bubble_centroid_velocity(self, i, comp):
        v = self.scripts[i](self.t)
        if v is None:
            raise PflbmError("pflbm_bubble_centroid_velocity", -4)
        return np.array([math.pi * R * R, 0.0, 30.0, self.yc(i), 0.0, v])

    def macroscopic(self, i):
        return {"phi": _Arr(disc(self.yc(i))[None])}


def case(name):
    prm = dict(nx=NX, ny=NY, rho=[1e-2, 1e-2, 1.0], g=1e-6, sigma13=1e-3, K=0.01, n=0.8)
    return dict(name=name, params=prm, C=disc()[None], u=None, p=None)


def test_peak_endings_and_report(monkeypatch):
    Scripted.scripts = [
        lambda t: 1e-3 - 1e-12 * (t - 5000) ** 2,                        # peaks on a plateau at 5,000
        lambda t: None if t >= 3000 else 1e-3,                            # becomes non-finite
        lambda t: 1e-4 * t / 1000,                                        # keeps accelerating
        lambda t: 0.02,                                                   # reaches the top wall
    ]
    out = sweep.run_sweep([case(f"c{i}") for i in range(4)], 10000, 1000, solver_factory=Scripted)
    a, b, c, d = out
    assert a["end"] == "max_steps" and a["peak_step"] == 5000
    assert a["plateau_change"] == pytest.approx(1e-6 / 1e-3, rel=1e-9)
    rep = a["report"]
    assert rep["U"] == pytest.approx(1e-3)
    assert rep["E"] == pytest.approx(1.0, abs=0.01) and rep["d_e"] == pytest.approx(2 * R, rel=1e-12)
    assert rep["Eo"] == pytest.approx(0.99 * 1e-6 * (2 * R) ** 2 / 1e-3, rel=1e-12)
    assert b["end"] == "nonfinite by step 3000" and b["report"] is None
    assert c["end"] == "max_steps" and c["report"] is None and "peak_step" not in c   # peak at the last sample
    assert d["end"] == "top_wall" and d["steps"] < 10000


@pytest.mark.parametrize("mobility, source, forcing", [("constant", "product", "mixed"),
                                                       ("variable", "link", "central")])
def test_table5_cases_carry_the_chosen_method_switches(mobility, source, forcing):
    cases = sweep.table5_cases(100.0, 1, mobility, source, forcing)
    assert len(cases) == 6
    for c in cases:
        p = c["params"]
        assert p["variable_mobility"] == (mobility == "variable")
        assert p["mobility_flux"] == (source == "link")
        assert p["hforce_cd"] == (forcing == "central")
        assert p["rho"][2] / p["rho"][0] == pytest.approx(100.0)


def test_reports_the_largest_sampled_velocity_also_for_a_diverged_case():
    """A case that turns non-finite still reports its largest sampled rise
    velocity and the step it was sampled at."""
    Scripted.scripts = [lambda t: None if t >= 4000 else 1e-6 * t]
    out = sweep.run_sweep([case("c0")], 10000, 1000, solver_factory=Scripted)
    assert out[0]["end"] == "nonfinite by step 4000"
    assert out[0]["max_vy"] == pytest.approx(3e-3) and out[0]["max_vy_step"] == 3000
