"""Pins of the open boundaries in x (Sec. 3.2, Table 2): a single-phase
power-law liquid enters through a velocity inlet (u = (u_in, 0), u_in = 0.1)
at x = 0 and leaves through a convective outflow at x = nx - 1, between walls
at rest.

- At the steady state the profile far from the inlet is the developed
  power-law profile of Eq. (34), u_x(y) = u_in (2n+1)/(n+1) (1 - |y/L|^((n+1)/n)),
  within Table 2's relative L2 error (tests/golden/table2_channel_erel.json,
  printed for the paper's 60 x 240 channel; checked here at half that size).
- Mass: the flux through every column equals the inflow u_in ny (the lattice
  is weakly compressible, so a boundary that lets less leave than enters
  shows up as a flux falling along x).
- The inlet nodes carry exactly u_in (the unknown populations are set so that
  the next velocity moment returns it).
"""
import json
import os

import numpy as np
import pytest

from oracle.pfo import run_case
from paper_2207_09431_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_channel_erel.json")


def developed(y, n, L, u_in):
    """Eq. (34): developed power-law profile between plates 2L apart carrying
    the mean velocity u_in."""
    return u_in * (2 * n + 1) / (n + 1) * (1 - np.abs(y / L) ** ((n + 1) / n))


@pytest.mark.parametrize("n", [0.5, 1.5])
def test_inlet_channel_reaches_the_developed_profile(n):
    ref = json.load(open(GOLDEN))
    bound = dict(zip(ref["n"], ref["E_rel"]))[n]
    nx, ny, u_in = 120, 30, 0.1
    case = inputs.channel_inlet(n, nx=nx, ny=ny, u_in=u_in)
    o = run_case(case, 6000)
    m = o.macroscopic()
    ux, uy = m["u"]
    L = ny / 2.0
    y = np.arange(ny) + 0.5 - L
    x = 3 * nx // 4
    err = np.linalg.norm(ux[:, x] - developed(y, n, L, u_in)) / np.linalg.norm(developed(y, n, L, u_in))
    assert err < bound, err
    flux = ux.sum(axis=0) / (u_in * ny)
    assert np.abs(flux - 1.0).max() < 1e-4, flux
    assert np.abs(ux[:, 0] - u_in).max() < 1e-12 and np.abs(uy[:, 0]).max() < 1e-12


def test_outflow_keeps_the_pressure_steady():
    """Once developed, the pressure field stops changing: the outflow releases
    what the inlet brings in (a plain convective condition on the whole
    populations would let the pressure grow by U dp/dx every step)."""
    case = inputs.channel_inlet(1.0, nx=120, ny=30)
    o = run_case(case, 5000)
    p0 = o.macroscopic()["p"]
    o.step(500)
    p1 = o.macroscopic()["p"]
    drop = p0[:, 0].mean() - p0[:, -1].mean()
    assert np.abs(p1 - p0).max() < 1e-6 * drop / 500 * 500, (np.abs(p1 - p0).max(), drop)


def test_inlet_and_outflow_keep_uniform_equilibrium_flow():
    """Uniform flow u = (u_in, 0) at p = 0 with its equilibrium populations is
    a fixed point of the interior scheme (no gradient, no force, and the
    collision leaves an equilibrium unchanged).  The velocity inlet must
    return exactly these populations at x = 0, including how its unknown
    populations share the momentum (the odd part of the equilibrium, Sec.
    3.2), and the convective outflow must return them at x = nx - 1; only the
    walls disturb the flow, one row per step.  After 3 steps every population
    of the rows at least 4 away from a wall, end columns included, equals its
    initial value."""
    nx, ny, u_in, steps = 24, 20, 0.1, 3
    case = inputs.channel_inlet(1.0, nx=nx, ny=ny, u_in=u_in)
    u = np.zeros((2, ny, nx))
    u[0] = u_in
    prm = dict(case["params"])
    from oracle.pfo import Oracle
    o = Oracle(prm)
    o.init_fields(case["C"], u, np.zeros((ny, nx)))
    g0, h0, _ = o.populations()
    o.step(steps)
    g1, h1, _ = o.populations()
    rows = slice(steps + 1, ny - steps - 1)
    scale = np.abs(g0).max()
    assert np.abs(g1[:, rows, :] - g0[:, rows, :]).max() <= 1e-14 * scale
    assert np.abs(h1[:, :, rows, :] - h0[:, :, rows, :]).max() <= 1e-14
    # the walls did disturb the rows next to them (the check above is not vacuous)
    assert np.abs(g1[:, 0, :] - g0[:, 0, :]).max() > 1e-6 * scale
