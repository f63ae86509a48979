"""Seeded synthetic inputs shared by the HIP path and the FP64 oracle.

This module holds only case definitions and random draws: the SplitMix64
stream, the tanh bubble profile used as the initial phase field
(Sec. 4.2, Eq. (42)), velocity noise, and the parameter presets of the
benchmark workloads.  It contains none of the lattice Boltzmann arithmetic
and imports neither the oracle nor the HIP binding; both sides receive the
identical host arrays produced here.

Coordinates: node (x, y) sits at integer position (x, y), x in [0, nx) is
periodic, y in [0, ny) is bounded by walls at y = -1/2 and y = ny - 1/2.
Fields are float64 arrays of shape (ny, nx) (row-major, x fastest).
"""
from __future__ import annotations

import copy
import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Draws offset+1 .. offset+n of the SplitMix64 stream seeded with `seed`.

    SplitMix64 (Steele, Lea, Flood 2014): state advances by the golden gamma,
    output is the variant-13 mix of the state.  Counter-based form: draw k is
    mix(seed + k*gamma), so any slice can be generated independently.
    """
    k = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK) + k * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, n: int, lo: float = 0.0, hi: float = 1.0, offset: int = 0) -> np.ndarray:
    """n doubles in [lo, hi) from the top 53 bits of SplitMix64 draws."""
    u = (splitmix64(seed, n, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return lo + (hi - lo) * u


def _bubble_box(nx: int, ny: int, cx: float, cy: float, r: float, xi: float):
    """Rows, columns and tanh profile of one bubble inside its box of
    half-width R + 20 (xi/2) + 1 (beyond it the float64 profile is exactly 0)."""
    half = r + 20.0 * (0.5 * xi) + 1.0
    if 2 * half >= nx:
        xs = np.arange(nx)
    else:
        xs = np.arange(int(np.floor(cx - half)), int(np.ceil(cx + half)) + 1) % nx
    ys = np.arange(max(0, int(np.floor(cy - half))), min(ny, int(np.ceil(cy + half)) + 1))
    y, x = np.meshgrid(ys.astype(np.float64), xs.astype(np.float64), indexing="ij")
    dx = x - cx
    dx = dx - nx * np.round(dx / nx)
    dist = np.sqrt(dx * dx + (y - cy) ** 2)
    return ys, xs, 0.5 - 0.5 * np.tanh((dist - r) / (0.5 * xi))


def bubble_field(nx: int, ny: int, bubbles, xi: float) -> np.ndarray:
    """Dispersed-phase concentration of circular bubbles with a tanh rim.

    Each bubble (cx, cy, R) contributes 0.5 - 0.5 tanh((r - R) / (xi/2)),
    the initial condition of Sec. 4.2 (Eq. (42)) with d_b = 2R.  Distances
    use the minimum image in the periodic x direction.  Contributions of
    separate bubbles are added and the sum is capped at 1.

    A contribution is evaluated only inside the bubble's box of half-width
    R + 20 (xi/2) + 1: beyond it the float64 tanh is exactly 1 and the term
    exactly 0, so the result equals the direct evaluation bit for bit.
    """
    c = np.zeros((ny, nx))
    for (cx, cy, r) in bubbles:
        ys, xs, prof = _bubble_box(nx, ny, cx, cy, r, xi)
        if len(ys):
            c[np.ix_(ys, xs)] += prof
    return np.minimum(c, 1.0)


def rest_pressure(nx: int, ny: int, bubbles, xi: float, sigma: float, rho_l: float, g: float) -> np.ndarray:
    """Pressure of the fluid at rest: the liquid's hydrostatic profile
    rho_l g (y_c - y) (y_c the mid-height) and, inside each bubble, the liquid
    pressure at the bubble's centre plus the Laplace jump sigma / R of a
    two-dimensional drop, blended with the bubble's own tanh profile.  The
    gas carries no hydrostatic gradient (its weight is negligible), which a
    plain hydrostatic start would impose on it.  Starting the bubbles at the
    liquid pressure instead (p = 0 inside) launches an acoustic transient that
    destabilises domains of 1024 x 1024 and more at density ratio 1000."""
    yc = 0.5 * (ny - 1)
    y = np.arange(ny, dtype=np.float64)[:, None]
    p = rho_l * g * (yc - y) * np.ones((1, nx))
    for (cx, cy, r) in bubbles:
        ys, xs, prof = _bubble_box(nx, ny, cx, cy, r, xi)
        if len(ys):
            pin = rho_l * g * (yc - cy) + sigma / r
            p[np.ix_(ys, xs)] += prof * (pin - rho_l * g * (yc - ys.astype(np.float64))[:, None])
    return p


def velocity_noise(nx: int, ny: int, seed: int, amp: float):
    """i.i.d. U[-amp, amp) noise for u_x then u_y, shape (2, ny, nx)."""
    v = uniform(seed, 2 * nx * ny, -amp, amp)
    return v.reshape(2, ny, nx)


def default_params(nx: int, ny: int) -> dict:
    """Parameter block with the ABI's field names (two-phase, Newtonian)."""
    return dict(
        nx=nx, ny=ny, n_h=1,
        rho=[1e-3, 1e-3, 1.0],       # rho_1 (gas), rho_2 (unused when n_h=1), rho_3 (liquid)
        nu=[1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0],
        powerlaw_comp=-1,            # component whose viscosity follows the power law, or -1
        K=0.1, n=1.0, nu_min=1e-4, nu_max=1.0,
        sigma12=1e-3, sigma13=1e-3, sigma23=1e-3, Lambda=0.0,
        xi=4.0, D0=4.0 / 300.0, variable_mobility=1,
        tau_h=0.5, g=0.0, fx=0.0,
        storage=0, store_h=0, hforce_cd=0, open_x=0, u_in=0.0, mobility_flux=0,
    )


def gravity_from_eotvos(eo: float, sigma: float, rho_l: float, rho_g: float, d: float) -> float:
    """g such that Eo = (rho_l - rho_g) g d^2 / sigma (Sec. 4.1, Eq. (40))."""
    return eo * sigma / ((rho_l - rho_g) * d * d)


def _case(params, C, u=None, p=None, name=""):
    return dict(name=name, params=params, C=np.ascontiguousarray(C, dtype=np.float64),
                u=None if u is None else np.ascontiguousarray(u, dtype=np.float64),
                p=None if p is None else np.ascontiguousarray(p, dtype=np.float64))


def hydrostatic_pressure(C, params: dict) -> np.ndarray:
    """Initial pressure of the liquid at rest under F_b = -rho g j:
    p(y) = rho_l g (y_c - y) with y_c the mid-height, the same in every column.
    Starting from p = 0 instead launches a pressure transient that a density
    ratio of 1000 does not survive for the larger g.  (Integrating the mixture
    density along each column is worse: columns that cross a bubble get a
    lower pressure below it, and the resulting horizontal pressure jump
    accelerates the gas of any bubble beneath.)"""
    C = np.asarray(C, dtype=np.float64)
    ny, nx = C.shape[-2:]
    rho_l = float(params["rho"][2])
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    return rho_l * float(params["g"]) * (0.5 * (ny - 1) - y)


# The density-ratio-1000 workloads below start from p = 0 (a quiescent
# start; the liquid settles into hydrostatic balance through a weak acoustic
# transient).  `rest_pressure` is the alternative start: it keeps a single
# bubble in a 1024 x 1024 box stable where p = 0 diverges after ~1,600 steps,
# but at density ratio 1000 neither start carries the 64-bubble 2048 x 4096
# domain past a few thousand steps (the oracle diverges with the GPU on the
# 1024 x 1024 case), and the faster initial gas transient of the rest start
# amplifies float32 rounding in the gas.  The density-ratio-100 long run uses
# the rest start.


def gravity_for_gas_mach(radius: float, density_ratio: float, mach: float = 0.01) -> float:
    """g whose buoyant acceleration of the gas, (rho_l/rho_g) g, reaches the
    velocity mach * c_s within one acoustic crossing R / c_s of the bubble."""
    cs = 1.0 / np.sqrt(3.0)
    return mach * cs * cs / (density_ratio * radius)


def rising_bubble_small(seed: int = 1, nx: int = 64, ny: int = 128, density_ratio: float = 100.0) -> dict:
    """Two-phase rising bubble, 64x128: R=8 at (32,32), xi=4, Newtonian
    liquid with tau_l = 0.8 (nu_l = 0.8/3), dynamic viscosity ratio 100
    (nu_g = 10 nu_l at density ratio 1000, kept at the lower density ratio),
    constant mobility scale 0.02, sigma = 1e-3, g from Eo = 10, velocity noise
    +-1e-4 and a hydrostatic initial pressure.  A bubble this small is stable
    at density ratio 100 with this scheme, not at 1000."""
    prm = default_params(nx, ny)
    nu_l = 0.8 / 3.0
    nu_g = 10.0 * nu_l
    rg = 1.0 / density_ratio
    prm.update(rho=[rg, rg, 1.0], nu=[nu_g, nu_g, nu_l], powerlaw_comp=-1, n=1.0,
               D0=0.02, variable_mobility=0,
               g=gravity_from_eotvos(10.0, 1e-3, 1.0, rg, 16.0))
    C = bubble_field(nx, ny, [(nx / 2.0, ny / 4.0, 8.0)], prm["xi"])[None]
    u = velocity_noise(nx, ny, seed, 1e-4)
    return _case(prm, C, u, hydrostatic_pressure(C, prm), f"rising_bubble_{nx}x{ny}")


def rising_bubble_terminal(nx: int = 128, ny: int = 512, radius: float = 24.0) -> dict:
    """A larger bubble of the small case's fluids (density ratio 100, Newtonian,
    nu_l = 0.8/3, nu_g = 10 nu_l, D0 = 0.02 constant mobility, sigma = 1e-3,
    g from Eo = 10 on d = 2R) at (nx/2, ny/5), hydrostatic p, no noise.  Its
    mean rise velocity levels off after ~6,000 steps and then drifts by
    ~0.1 % per 1,000 steps as the bubble slowly dissolves (constant mobility),
    which gives the terminal-velocity comparison a plateau."""
    prm = default_params(nx, ny)
    nu_l = 0.8 / 3.0
    rg = 1.0 / 100.0
    prm.update(rho=[rg, rg, 1.0], nu=[10.0 * nu_l, 10.0 * nu_l, nu_l], powerlaw_comp=-1, n=1.0,
               D0=0.02, variable_mobility=0, g=gravity_from_eotvos(10.0, 1e-3, 1.0, rg, 2.0 * radius))
    C = bubble_field(nx, ny, [(nx / 2.0, ny / 5.0, radius)], prm["xi"])[None]
    return _case(prm, C, None, hydrostatic_pressure(C, prm), f"rising_bubble_terminal_{nx}x{ny}_R{radius:g}")


def static_bubble(nx: int = 96, ny: int = 96, radius: float = 25.0, density_ratio: float = 1000.0,
                  sigma: float = 1e-4, variable_mobility: int = 0) -> dict:
    """Bubble at rest in the middle of the box, no gravity."""
    prm = default_params(nx, ny)
    rg = 1.0 / density_ratio
    prm.update(rho=[rg, rg, 1.0], nu=[1.0 / 6.0] * 3, sigma12=sigma, sigma13=sigma, sigma23=sigma,
               variable_mobility=variable_mobility, g=0.0)
    C = bubble_field(nx, ny, [(nx / 2.0, ny / 2.0, radius)], prm["xi"])[None]
    return _case(prm, C, None, None, f"static_bubble_{nx}x{ny}_R{radius}")


def powerlaw_bubble(n: float = 0.5, eo: float = 10.0, nx: int = 200, ny: int = 400, d: float = 50.0,
                    density_ratio: float = 1000.0, K: float = 0.1, mach: float = 0.01) -> dict:
    """Single bubble (diameter d, centre (nx/2, 0.6 nx), Eq. (42)) rising in
    a power-law liquid, K and n given, nu in [1e-4, 1], gas nu = c_s^2 * 0.5
    (tau_d = 0.5 as in the paper's Table 5), constant mobility xi/300,
    g from `gravity_for_gas_mach` and sigma from Eo."""
    prm = default_params(nx, ny)
    rg = 1.0 / density_ratio
    g = gravity_for_gas_mach(d / 2.0, density_ratio, mach)
    sigma = (1.0 - rg) * g * d * d / eo
    prm.update(rho=[rg, rg, 1.0], nu=[1.0 / 6.0, 1.0 / 6.0, 1.0], powerlaw_comp=2,
               K=K, n=n, nu_min=1e-4, nu_max=1.0, variable_mobility=0,
               sigma12=sigma, sigma13=sigma, sigma23=sigma, g=g)
    C = bubble_field(nx, ny, [(nx / 2.0, 0.6 * nx, d / 2.0)], prm["xi"])[None]
    return _case(prm, C, None, None, f"powerlaw_bubble_{nx}x{ny}_n{n:.3f}_Eo{eo:.2f}")



# Table 5 (Sec. 4.3): power-law index n, consistency k, gravity g, surface
# tension sigma of the six shear-thinning cases (d_b = L/4 = 50, tau_d = 0.5)
TABLE5_FLUIDS = ((0.5, 1e-4, 5e-7, 2.61e-6), (0.5, 1e-4, 5e-7, 2.61e-5), (0.5, 2e-4, 5e-7, 5e-4),
                 (0.6, 5e-4, 2e-7, 2.61e-5), (0.63, 5e-4, 2e-7, 2.61e-5), (0.8, 1e-2, 5e-7, 2.61e-5))


def grid_scaled(n: float, k: float, g: float, sigma: float, f: float):
    """Power-law consistency, gravity and surface tension on a lattice f times
    finer with the same Re, Eo and Mo (Eqs. (38)-(40)): lattice velocities
    scale by 1/f and lengths by f, so k * f^(2n-2), g / f^3, sigma / f
    (for n = 0.5 this is the progression of Table 4's grids)."""
    return k * f ** (2.0 * n - 2.0), g / f ** 3, sigma / f


def shear_thinning_sweep(density_ratio: float = 800.0, scale: int = 1) -> list:
    """The six bubbles of Table 5: d = L/4 at (L/2, 0.6 L) (Eq. (42)) on an
    L x 2L lattice, L = 200 * scale, in a power-law liquid (rho_l = 1) with
    the printed n, k, g and sigma (scaled by `grid_scaled` when scale > 1);
    gas nu = c_s^2 * 0.5 (tau_d = 0.5), nu in [1e-4, 1], constant mobility
    xi/300, the bubble started at its rest pressure.  The paper's density
    ratio is 800."""
    out = []
    nx, ny = 200 * scale, 400 * scale
    d = nx / 4.0
    for i, (n, k0, g0, sigma0) in enumerate(TABLE5_FLUIDS):
        k, g, sigma = grid_scaled(n, k0, g0, sigma0, scale)
        prm = default_params(nx, ny)
        rg = 1.0 / density_ratio
        prm.update(rho=[rg, rg, 1.0], nu=[1.0 / 6.0, 1.0 / 6.0, 1.0], powerlaw_comp=2,
                   K=k, n=n, nu_min=1e-4, nu_max=1.0, variable_mobility=0,
                   sigma12=sigma, sigma13=sigma, sigma23=sigma, g=g)
        b = [(nx / 2.0, 0.6 * nx, d / 2.0)]
        C = bubble_field(nx, ny, b, prm["xi"])[None]
        p = rest_pressure(nx, ny, b, prm["xi"], sigma, 1.0, g)
        out.append(_case(prm, C, None, p, f"table5_case{i + 1}_{nx}x{ny}_ratio{density_ratio:g}"))
    return out


def three_component(variable_mobility: int = 0, nx: int = 256, ny: int = 512,
                    density_ratio: float = 1000.0) -> dict:
    """Three components: C1 bubble R=40 at (128,160), C2 bubble R=25 at
    (128,330) above it, liquid C3 power law n=0.7, K=0.1, both dispersed
    phases rho = 1/density_ratio (1e-3 by default), nu = 1/6,
    sigma_ij = 1e-4, Lambda = 0; g from the gas-Mach rule at ratio 1000."""
    prm = default_params(nx, ny)
    sx, sy = nx / 256.0, ny / 512.0
    g = gravity_for_gas_mach(40.0, 1000.0, 0.01)
    rg = 1.0 / density_ratio
    prm.update(n_h=2, rho=[rg, rg, 1.0], nu=[1.0 / 6.0, 1.0 / 6.0, 1.0], powerlaw_comp=2,
               K=0.1, n=0.7, nu_min=1e-4, nu_max=1.0, variable_mobility=variable_mobility,
               sigma12=1e-4, sigma13=1e-4, sigma23=1e-4, g=g)
    s = min(sx, sy)
    b1, b2 = (128.0 * sx, 160.0 * sy, 40.0 * s), (128.0 * sx, 330.0 * sy, 25.0 * s)
    c1 = bubble_field(nx, ny, [b1], prm["xi"])
    c2 = bubble_field(nx, ny, [b2], prm["xi"])
    C = np.stack([c1, c2])
    return _case(prm, C, None, None, f"three_component_{nx}x{ny}")


def bubble_droplet(variable_mobility: int = 1, nx: int = 200, ny: int = 400, tau3: float = 0.5,
                   r_bubble: float = 20.0, r_drop: float = 25.0, gap: float = 10.0, hforce_cd: int = 1) -> dict:
    """The three-component system of Sec. 3.1 (Table 1): a light bubble
    (component 2, rho_2 = 0.01) rising under g = 1e-6 towards a droplet of
    the liquid's density (component 1, rho_1 = rho_3 = 1) in the liquid
    (component 3), all sigma_ij = 1e-4, tau_1/tau_3 = tau_2/tau_3 = 2, on a
    200 x 400 lattice.  The paper shows the initial state only as a figure and
    gives no tau_3; here tau_3 = 1/2 (nu = c_s^2 tau), the droplet (radius
    r_drop) is centred at (nx/2, ny/2) and the bubble (radius r_bubble) on the
    same vertical line `gap` lattice units below it.  D0 = xi/300 (Sec. 2.1).
    hforce_cd selects central differences for grad C_i in the hbar forcing,
    the reading under which variable mobility is stable."""
    prm = default_params(nx, ny)
    nu3 = tau3 / 3.0
    prm.update(n_h=2, rho=[1.0, 0.01, 1.0], nu=[2.0 * nu3, 2.0 * nu3, nu3], powerlaw_comp=-1, n=1.0,
               sigma12=1e-4, sigma13=1e-4, sigma23=1e-4, Lambda=0.0, variable_mobility=variable_mobility,
               D0=prm["xi"] / 300.0, g=1e-6, hforce_cd=hforce_cd)
    yd = ny / 2.0
    yb = yd - r_drop - gap - r_bubble
    c1 = bubble_field(nx, ny, [(nx / 2.0, yd, r_drop)], prm["xi"])
    c2 = bubble_field(nx, ny, [(nx / 2.0, yb, r_bubble)], prm["xi"])
    return _case(prm, np.stack([c1, c2]), None, None,
                 f"bubble_droplet_{nx}x{ny}_{'variable' if variable_mobility else 'constant'}_mobility")


def place_bubbles(nx: int, ny: int, count: int, rmin: float, rmax: float, xi: float, seed: int,
                  max_draws: int = 200000):
    """Rejection sampling of non-overlapping bubbles: centre gap >= R1+R2+2xi,
    distance to each wall >= R+2xi.  Draws come from one SplitMix64 stream."""
    out = []
    k = 0
    while len(out) < count:
        if k >= max_draws:
            raise RuntimeError("could not place bubbles")
        r, cx, cy = uniform(seed, 3, 0.0, 1.0, offset=3 * k)
        k += 1
        r = rmin + (rmax - rmin) * r
        cx = cx * nx
        cy = r + 2 * xi + cy * (ny - 2 * (r + 2 * xi))
        ok = True
        for (bx, by, br) in out:
            dx = cx - bx
            dx -= nx * round(dx / nx)
            if (dx * dx + (cy - by) ** 2) < (r + br + 2 * xi) ** 2:
                ok = False
                break
        if ok:
            out.append((cx, cy, r))
    return out


LARGE_RMIN, LARGE_RMAX = 25.0, 40.0


def large_domain_params(nx: int = 2048, ny: int = 4096, storage: int = 0, density_ratio: float = 1000.0) -> dict:
    """Power-law liquid n=0.6, K=0.1, nu in [1e-4, 1], density ratio 1000 (or
    as given), sigma = 1e-4, g from `gravity_for_gas_mach` at the largest
    radius."""
    prm = default_params(nx, ny)
    rg = 1.0 / density_ratio
    prm.update(rho=[rg, rg, 1.0], nu=[1.0 / 6.0, 1.0 / 6.0, 1.0], powerlaw_comp=2,
               K=0.1, n=0.6, nu_min=1e-4, nu_max=1.0, variable_mobility=0,
               sigma12=1e-4, sigma13=1e-4, sigma23=1e-4,
               g=gravity_for_gas_mach(LARGE_RMAX, density_ratio, 0.01), storage=storage)
    return prm


def _at_rest(prm: dict, bubbles) -> np.ndarray:
    return rest_pressure(prm["nx"], prm["ny"], bubbles, prm["xi"], prm["sigma12"], prm["rho"][2], prm["g"])


def many_bubbles(nx: int = 2048, ny: int = 4096, count: int = 64, seed: int = 5, storage: int = 0,
                 density_ratio: float = 1000.0, at_rest: bool = False) -> dict:
    """Large single domain with `count` non-overlapping seeded bubbles,
    R ~ U[25, 40], in the power-law liquid of `large_domain_params`, starting
    from p = 0 or (at_rest) from the pressure at rest."""
    prm = large_domain_params(nx, ny, storage, density_ratio)
    bubbles = place_bubbles(nx, ny, count, LARGE_RMIN, LARGE_RMAX, prm["xi"], seed)
    C = bubble_field(nx, ny, bubbles, prm["xi"])[None]
    tag = ("" if density_ratio == 1000.0 else f"_ratio{density_ratio:g}") + ("_rest" if at_rest else "")
    case = _case(prm, C, None, _at_rest(prm, bubbles) if at_rest else None, f"many_bubbles_{nx}x{ny}_{count}{tag}")
    case["bubbles"] = bubbles
    return case


def many_bubbles_crop(nx: int = 2048, ny: int = 4096, count: int = 64, seed: int = 5,
                      cw: int = 256, ch: int = 512, storage: int = 0) -> dict:
    """A cw x ch window of `many_bubbles`, as its own domain with the same
    physical parameters: the window is centred on the first placed bubble
    (clamped to the domain) and keeps the bubbles lying fully inside it."""
    prm = large_domain_params(cw, ch, storage)
    bubbles = place_bubbles(nx, ny, count, LARGE_RMIN, LARGE_RMAX, prm["xi"], seed)
    bx, by, _ = bubbles[0]
    x0 = int(min(max(np.floor(bx) - cw // 2, 0), nx - cw))
    y0 = int(min(max(np.floor(by) - ch // 2, 0), ny - ch))
    inside = [(x - x0, y - y0, r) for (x, y, r) in bubbles
              if x - r - prm["xi"] >= x0 and x + r + prm["xi"] < x0 + cw
              and y - r - prm["xi"] >= y0 and y + r + prm["xi"] < y0 + ch]
    C = bubble_field(cw, ch, inside, prm["xi"])[None]
    case = _case(prm, C, None, None, f"many_bubbles_crop_{cw}x{ch}")
    case["bubbles"] = inside
    case["origin"] = (x0, y0)
    return case


def batch_sweep(count_per_size: int = 16, seed: int = 4, sizes=((150, 300), (200, 400), (300, 600)),
                density_ratio: float = 1000.0):
    """Uneven batch: `count_per_size` cases of each size, n ~ U[0.5,1.5],
    Eo ~ U[1,100], d = width/5, density ratio 1000 unless given (the same
    draws of n and Eo at any ratio)."""
    cases = []
    k = 0
    for (nx, ny) in sizes:
        for _ in range(count_per_size):
            n, eo = uniform(seed, 2, 0.0, 1.0, offset=2 * k)
            k += 1
            n = 0.5 + n
            eo = 1.0 + 99.0 * eo
            c = powerlaw_bubble(n=n, eo=eo, nx=nx, ny=ny, d=nx / 5.0, density_ratio=density_ratio)
            c["name"] = f"batch_{nx}x{ny}_{k}"
            cases.append(c)
    return cases


def channel(n: float, ny: int = 32, nx: int = 5, fx: float = 1e-6, K: float = 0.01,
            nu_min: float = 1e-3, nu_max: float = 1.0) -> dict:
    """Single-phase power-law liquid between walls, driven by a body force
    along x (liquid only: C1 = 0)."""
    prm = default_params(nx, ny)
    prm.update(rho=[1.0, 1.0, 1.0], nu=[1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0], powerlaw_comp=2,
               K=K, n=n, nu_min=nu_min, nu_max=nu_max, g=0.0, fx=fx)
    C = np.zeros((1, ny, nx))
    return _case(prm, C, None, None, f"channel_n{n}")


def channel_inlet(n: float, nx: int = 240, ny: int = 60, u_in: float = 0.1, nu_wall: float = 0.2,
                  nu_min: float = 1e-3, nu_max: float = 5.0) -> dict:
    """The single-phase power-law channel of Sec. 3.2 (Table 2): length nx
    along x with a velocity inlet u_in at x = 0 and a convective outflow at
    x = nx - 1, walls at rest below and above (width ny), the liquid
    (component 3) everywhere, no body force.  The paper gives no consistency
    K or truncation; here K makes the viscosity at the wall of the developed
    profile nu_wall, K = nu_wall / gdot_w^(n-1) with the developed wall shear
    rate gdot_w = u_in (2n+1) / (n L), L = ny/2, and nu is limited to
    [nu_min, nu_max], outside most of the profile."""
    prm = default_params(nx, ny)
    L = ny / 2.0
    gw = u_in * (2.0 * n + 1.0) / (n * L)
    K = nu_wall / gw ** (n - 1.0)
    prm.update(rho=[1.0, 1.0, 1.0], nu=[1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0], powerlaw_comp=2,
               K=K, n=n, nu_min=nu_min, nu_max=nu_max, g=0.0, fx=0.0, open_x=1, u_in=u_in)
    C = np.zeros((1, ny, nx))
    return _case(prm, C, None, None, f"channel_inlet_n{n}_{nx}x{ny}")


def layered_flow(n3: float, lam: float, ny: int = 200, nx: int = 5, nu1: float = 1.0 / 6.0,
                 fx: float = 1e-6, nu_min: float = 1e-3, nu_max: float = 1.0, sigma: float = 5e-4,
                 xi: float = 4.0) -> dict:
    """Two-layer flow between the walls (Sec. 3.3, Fig. 6): component 3, a
    power-law liquid of index n3, fills |y - y_c| < Y_i = ny/4 around the
    channel centre y_c; component 1, Newtonian with nu1, fills the rest
    (tanh rims of width xi); C2 = 0.  Equal densities (rho = 1), sigma_13 =
    sigma, constant mobility, body force fx along the periodic x.  The
    consistency ratio lam = K3 / (rho_1 nu1) is the paper's lambda^P
    (lambda for n3 = 1)."""
    prm = default_params(nx, ny)
    K3 = lam * nu1
    prm.update(rho=[1.0, 1.0, 1.0], nu=[nu1, nu1, nu1], powerlaw_comp=2, K=K3, n=n3,
               nu_min=nu_min, nu_max=nu_max, sigma12=sigma, sigma13=sigma, sigma23=sigma, xi=xi,
               variable_mobility=0, g=0.0, fx=fx)
    H = ny / 2.0
    s = np.abs(np.arange(ny) + 0.5 - H)          # node distance from the centre line
    c1 = 0.5 + 0.5 * np.tanh((s - H / 2.0) / (xi / 2.0))
    C = np.repeat(c1[:, None], nx, axis=1)[None]
    return _case(prm, C, None, None, f"layered_n{n3}_lam{lam:g}_{nx}x{ny}")


def clone(case: dict) -> dict:
    return copy.deepcopy(case)
