"""Drag coefficient and dimensionless numbers of a rising bubble (Sec. 4.1,
Eqs. (37)-(41)), from the diagnostics the GPU path returns.

Host post-processing of a few scalars and one copied-back field; the time
stepping itself runs only in the HIP library.  Lattice units throughout
(lengths in nodes, time in steps, rho_l the liquid's density).

Readings of the paper's definitions:
- `d` in C_D and Re, Mo, Eo is the bubble's diameter; the paper's d_e comes
  from a three-dimensional volume, which a two-dimensional lattice does not
  have, so the equivalent diameter here is that of the circle with the
  bubble's area, sqrt(4 A / pi), A = sum of the gas fraction C over the
  nodes.  The Eo values of Table 6 follow from the initial diameter d_b with
  rho_l in place of rho_l - rho_g; `eotvos` takes the density difference as
  an argument so either form can be formed.
- E is the ratio of the vertical to the horizontal diameter of the C = 1/2
  contour, measured on the lines through the bubble's centroid.
- Li et al.'s correlation (Eq. (41)) carries (1 - E)^0.681, which is real
  only for E <= 1 (Table 7 lists E < 1); for E > 1 the deformation factor is
  taken as 1 (the value at E = 1).
"""
from __future__ import annotations

import math

import numpy as np


def drag_coefficient(d: float, g: float, rho_l: float, rho_g: float, U: float) -> float:
    """Drag coefficient at terminal velocity U: buoyancy of the bubble balanced
    by drag, C_D = 4 d g (rho_l - rho_g) / (3 rho_l U^2) (Eq. (37))."""
    return 4.0 * d * g * (rho_l - rho_g) / (3.0 * rho_l * U * U)


def reynolds(rho_l: float, U: float, d: float, k: float, n: float) -> float:
    """Power-law Reynolds number rho_l U^(2-n) d^n / k (Eq. (38)); for n = 1
    it is U d / nu with nu = k / rho_l."""
    return rho_l * U ** (2.0 - n) * d ** n / k


def morton(g: float, drho: float, rho_l: float, sigma: float, k: float, U: float, d: float, n: float) -> float:
    """Power-law Morton number g drho mu_eff^4 / (rho_l^2 sigma^3) with the
    effective viscosity mu_eff = k (U/d)^(n-1) (Eq. (39))."""
    mu_eff = k * (U / d) ** (n - 1.0)
    return g * drho * mu_eff ** 4 / (rho_l * rho_l * sigma ** 3)


def eotvos(drho: float, g: float, d: float, sigma: float) -> float:
    """Eotvos number drho g d^2 / sigma (Eq. (40))."""
    return drho * g * d * d / sigma


def li_drag_coefficient(Re: float, n: float, E: float) -> float:
    """Li et al.'s drag correlation for a bubble in a shear-thinning liquid
    (Eq. (41)): 16/Re (1 + 0.43 Re^0.44) (1 + 3.868 n^0.7528 (1 - E)^0.681),
    the deformation factor taken as 1 for E >= 1."""
    deform = 1.0 + 3.868 * n ** 0.7528 * (1.0 - E) ** 0.681 if E < 1.0 else 1.0
    return 16.0 / Re * (1.0 + 0.43 * Re ** 0.44) * deform


def li_terminal_velocity(d: float, g: float, rho_l: float, rho_g: float, k: float, n: float, E: float) -> float:
    """Terminal velocity predicted by the correlation: the U at which the drag
    coefficient of the force balance (Eq. (37)) equals Li et al.'s (Eq. (41))
    with Re(U) of Eq. (38) -- Table 7's "Li et al." column.  The balance
    falls like U^-2 and the correlation at most like U^-(2-n) with n > 0, so
    their ratio is monotone and the root is unique; found by bisection in
    log U."""
    def f(U):
        return math.log(drag_coefficient(d, g, rho_l, rho_g, U)) - \
            math.log(li_drag_coefficient(reynolds(rho_l, U, d, k, n), n, E))
    lo, hi = 1e-12, 1e3
    if not (f(lo) > 0.0 > f(hi)):
        raise ValueError("no terminal velocity in [1e-12, 1e3]")
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
        if hi / lo - 1.0 < 1e-14:
            break
    return math.sqrt(lo * hi)


def dimensionless_velocity(U: float, g: float, d: float) -> float:
    """Rise velocity scaled by sqrt(g d) (Sec. 4.2)."""
    return U / math.sqrt(g * d)


def dimensionless_height(y: float, L: float) -> float:
    """Centroid height scaled by the domain height 2L of the L x 2L box
    (Sec. 4.2)."""
    return y / (2.0 * L)


def equivalent_diameter(area: float) -> float:
    """Diameter of the circle of the given area (the two-dimensional form of
    the paper's volume-equivalent diameter)."""
    return math.sqrt(4.0 * area / math.pi)


def _crossing(profile: np.ndarray, centre: int, step: int) -> float:
    """Distance from index `centre` along `profile` (in direction `step`) to
    where the profile first falls to 1/2, linearly interpolated; the profile
    is periodic (indices wrap)."""
    m = profile.shape[0]
    prev = profile[centre % m]
    for s in range(1, m):
        cur = profile[(centre + step * s) % m]
        if cur <= 0.5:
            return (s - 1) + (prev - 0.5) / (prev - cur)
        prev = cur
    raise ValueError("profile never falls to 1/2")


def bubble_shape(phi: np.ndarray, xc: float, yc: float) -> dict:
    """Horizontal and vertical diameters of the C = 1/2 contour of a bubble
    (gas fraction `phi`, shape (ny, nx)) on the grid lines nearest its
    centroid (xc, yc), with the aspect ratio E = vertical / horizontal.
    x wraps (periodic); a bubble must not touch the walls."""
    phi = np.asarray(phi, dtype=np.float64)
    ny, nx = phi.shape
    i, j = int(round(xc)) % nx, int(round(yc))
    if not (0 <= j < ny) or phi[j, i] <= 0.5:
        raise ValueError("the centroid is not inside the bubble")
    row, col = phi[j, :], phi[:, i]
    # offsets of the grid line from the centroid are second order for the
    # diameter; the contour is measured from the node at the centroid
    horiz = _crossing(row, i, 1) + _crossing(row, i, -1)
    vert = _crossing(col, j, 1) + _crossing(col, j, -1)
    return {"horizontal": horiz, "vertical": vert, "E": vert / horiz}


def bubble_report(diag, phi: np.ndarray, rho_l: float, rho_g: float, g: float, sigma: float,
                  k: float, n: float, U: float | None = None) -> dict:
    """Dimensionless numbers of a bubble from the six diagnostics of the
    centroid reduction (sum C, sum of C above 1/2, x_c, y_c, mean u_x, mean
    u_y; Eqs. (43)-(44)) and its gas-fraction field: U (the mean rise
    velocity unless given), d_e, E, Re, Eo, Mo, the drag coefficient of the
    force balance, the correlation's drag coefficient and terminal velocity
    at the measured E, and the scaled velocity U / sqrt(g d_e) and height
    y_c / (2L) of Sec. 4.2 (L the lattice width)."""
    mass, _, xc, yc, _, uy = (float(v) for v in diag)
    U = uy if U is None else float(U)
    de = equivalent_diameter(mass)
    shape = bubble_shape(phi, xc, yc)
    drho = rho_l - rho_g
    Re = reynolds(rho_l, U, de, k, n)
    return {
        "U": U, "d_e": de, "E": shape["E"], "Re": Re,
        "Eo": eotvos(drho, g, de, sigma),
        "Mo": morton(g, drho, rho_l, sigma, k, U, de, n),
        "C_D": drag_coefficient(de, g, rho_l, rho_g, U),
        "C_D_li": li_drag_coefficient(Re, n, shape["E"]),
        "U_li": li_terminal_velocity(de, g, rho_l, rho_g, k, n, shape["E"]),
        "U_star": dimensionless_velocity(U, g, de),
        "y_star": dimensionless_height(yc, phi.shape[1]),
    }
