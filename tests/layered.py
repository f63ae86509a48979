"""Closed form of the two-layer flow of Sec. 3.3 (Fig. 6), shared by the
oracle and GPU tests.

A body force G along the periodic x drives two layers between the walls at
distance H = ny/2 from the centre line: component 3 (truncated power law,
consistency K3, index n3) for |y| < Y_i = H/2 and component 1 (Newtonian,
nu1) outside, both of density 1.  The stress is tau_xy = -G y in both, so the
local shear rate solves nu(gdot) gdot = G |y| with the law of the layer at
|y|, and u(y) = int_|y|^H gdot(s) ds.  Without truncation this is the
paper's layered profile (Sec. 3.3, Eq. (36)): inside, the power-law part
n3/(n3+1) (G/K3)^(1/n3) (Y_i^((n3+1)/n3) - |y|^((n3+1)/n3)) plus the outer
layer's velocity at Y_i; outside, n1/(n1+1) (G/mu1)^(1/n1)
(H^((n1+1)/n1) - |y|^((n1+1)/n1)).  (The printed equation writes Y_i where
the outer layer's terms need the half-height H; with Y_i the outer layer
would move backwards.)
"""
import numpy as np


def shear_rate(stress, K, n, nu_min, nu_max):
    """Solve clamp(K g^(n-1), nu_min, nu_max) g = stress for g >= 0."""
    if stress <= 0:
        return 0.0
    g = (stress / K) ** (1.0 / n)
    nu = K * g ** (n - 1.0)
    if nu > nu_max:
        return stress / nu_max
    if nu < nu_min:
        return stress / nu_min
    return g


def two_layer_profile(ny, G, K3, n3, nu1, nu_min, nu_max, fine=20000):
    """u_x at the node rows y = 0..ny-1 (walls at -1/2 and ny - 1/2): the
    trapezoid rule on each layer separately (the shear rate jumps at Y_i)."""
    H = ny / 2.0
    Yi = H / 2.0
    so = np.linspace(Yi, H, fine + 1)                     # outer layer
    go = G * so / nu1
    Uo = np.concatenate([np.cumsum((0.5 * (go[1:] + go[:-1]) * np.diff(so))[::-1])[::-1], [0.0]])
    si = np.linspace(0.0, Yi, fine + 1)                   # inner layer, from u(Y_i) = Uo[0]
    gi = np.array([shear_rate(G * v, K3, n3, nu_min, nu_max) for v in si])
    Ui = Uo[0] + np.concatenate([np.cumsum((0.5 * (gi[1:] + gi[:-1]) * np.diff(si))[::-1])[::-1], [0.0]])
    ys = np.abs(np.arange(ny) + 0.5 - H)
    return np.where(ys < Yi, np.interp(ys, si, Ui), np.interp(ys, so, Uo))


def force_for_peak(umax, ny, K3, n3, nu1, nu_min, nu_max):
    """Body force whose closed-form centre velocity is umax (bisection on a
    log scale; the centre velocity grows monotonically with G)."""
    lo, hi = 1e-14, 1e-2
    for _ in range(120):
        mid = np.sqrt(lo * hi)
        if two_layer_profile(ny, mid, K3, n3, nu1, nu_min, nu_max, 4000).max() > umax:
            hi = mid
        else:
            lo = mid
    return np.sqrt(lo * hi)
