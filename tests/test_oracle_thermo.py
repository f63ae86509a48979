"""Pins of the oracle's ternary thermodynamics (Sec. 2.1, Eqs. (2)-(7)).

- Two-phase reduction (C2 = 0, equal sigma): mu_1 is the binary Cahn-Hilliard
  potential (12 sigma/xi) C(1-C)(1-2C) - (3/4) xi sigma lap C, mu_2 = 0,
  mu_3 = -mu_1 (derived by hand from Eqs. (3), (5)).
- Projection identity: sum_i mu_i / Sigma_i = 0 for any state.
- Thermodynamic consistency: for a variation with sum_i dC_i = 0,
  sum_i mu_i^bulk dC_i = (12/xi) dE0, checked against finite differences of
  the bulk energy E0.
- The tanh profile C = 1/2 + 1/2 tanh(2z/xi) makes the continuum mu vanish.
"""
import numpy as np
import pytest

from oracle import pfo
from paper_2207_09431_amd import inputs


def params(s12=1e-3, s13=1e-3, s23=1e-3, lam=0.0, xi=4.0):
    p = inputs.default_params(8, 8)
    p.update(sigma12=s12, sigma13=s13, sigma23=s23, Lambda=lam, xi=xi)
    return p


@pytest.mark.parametrize("c", [0.0, 0.1, 0.37, 0.5, 0.83, 1.0, 1.02])
@pytest.mark.parametrize("lap", [0.0, 0.013])
def test_binary_reduction(c, lap):
    sig, xi = 2e-3, 5.0
    p = params(sig, sig, sig, 0.0, xi)
    mu = pfo.chem_potential(p, [c, 0.0, 1.0 - c], [lap, 0.0, -lap])
    ref = 12 * sig / xi * c * (1 - c) * (1 - 2 * c) - 0.75 * xi * sig * lap
    assert abs(mu[0] - ref) < 1e-15
    assert abs(mu[1]) < 1e-15
    assert abs(mu[2] + ref) < 1e-15


def test_projection_identity():
    rng = np.random.default_rng(0)
    for _ in range(50):
        s = rng.uniform(1e-4, 3e-3, 3)
        s = s + 0.5 * s.max()  # keep every Sigma_i positive
        p = params(s[0], s[1], s[2], rng.uniform(0, 1e-3))
        S = np.array([s[0] + s[1] - s[2], s[0] + s[2] - s[1], s[1] + s[2] - s[0]])
        c = rng.dirichlet([1, 1, 1])
        lap = rng.normal(0, 1e-2, 3)
        lap[2] = -lap[0] - lap[1]
        mu = pfo.chem_potential(p, c, lap)
        assert abs((mu / S).sum()) < 1e-14 * max(1.0, np.abs(mu / S).max())


def test_bulk_consistency_with_energy():
    rng = np.random.default_rng(1)
    for _ in range(30):
        s = rng.uniform(5e-4, 2e-3, 3)
        s = s + 0.5 * s.max()
        lam = rng.uniform(0, 2e-3)
        xi = 4.0
        p = params(s[0], s[1], s[2], lam, xi)
        c = rng.dirichlet([2, 2, 2])
        dC = rng.normal(size=3)
        dC -= dC.mean()
        eps = 1e-6
        dE = (pfo.bulk_energy(p, *(c + eps * dC)) - pfo.bulk_energy(p, *(c - eps * dC))) / (2 * eps)
        mu = pfo.chem_potential(p, c, [0.0, 0.0, 0.0])
        assert abs(mu @ dC - 12.0 / xi * dE) < 1e-7 * abs(12.0 / xi * dE) + 1e-15


def test_bulk_energy_binary_limit():
    sig = 1.3e-3
    p = params(sig, sig, sig)
    for c in np.linspace(0, 1, 11):
        assert abs(pfo.bulk_energy(p, c, 0.0, 1 - c) - sig * c * c * (1 - c) ** 2) < 1e-18


def test_ternary_with_absent_component_is_binary():
    # C1 = 0: components 2 and 3 form a binary pair; with equal sigma_ij the
    # potential of component 2 is the binary one with sigma_23
    sig = 1e-3
    p = params(sig, sig, sig)
    for c in [0.2, 0.5, 0.9]:
        mu = pfo.chem_potential(p, [0.0, c, 1 - c], [0.0, 0.01, -0.01])
        ref = 12 * sig / 4.0 * c * (1 - c) * (1 - 2 * c) - 0.75 * 4.0 * sig * 0.01
        assert abs(mu[1] - ref) < 1e-15
        assert abs(mu[0]) < 1e-15


def test_tanh_profile_is_continuum_equilibrium():
    # mu(z) = (12 s/xi) C(1-C)(1-2C) - (3/4) xi s C'' vanishes for C = 1/2 + 1/2 tanh(2 z / xi)
    sig, xi = 1e-3, 4.0
    p = params(sig, sig, sig, 0.0, xi)
    for z in np.linspace(-6, 6, 13):
        t = np.tanh(2 * z / xi)
        c = 0.5 + 0.5 * t
        cpp = -(4.0 / xi ** 2) * t * (1 - t * t)    # d^2/dz^2 of 1/2 + 1/2 tanh(2z/xi)
        mu = pfo.chem_potential(p, [c, 0.0, 1 - c], [cpp, 0.0, -cpp])
        assert abs(mu[0]) < 1e-17


def _energy_sum_form(S, lam, c):
    """E0 written per component: sum_i (Sigma_i / 2) C_i^2 (1 - C_i)^2 +
    Lambda C1^2 C2^2 C3^2.  Equal to Eq. (3) whenever C1 + C2 + C3 = 1
    (expand (1 - C_i)^2 = (C_j + C_k)^2 and use Sigma_i + Sigma_j =
    2 sigma_ij); it shares no term-by-term structure with the pairwise form."""
    c = np.asarray(c, dtype=np.float64)
    return float(sum(0.5 * S[i] * c[i] ** 2 * (1.0 - c[i]) ** 2 for i in range(3))
                 + lam * (c[0] * c[1] * c[2]) ** 2)


def _random_ternary(rng):
    s = rng.uniform(5e-4, 2e-3, 3)
    s = s + 0.5 * s.max()                 # every Sigma_i > 0
    S = np.array([s[0] + s[1] - s[2], s[0] + s[2] - s[1], s[1] + s[2] - s[0]])
    return s, S, rng.uniform(1e-4, 3e-3)


def test_ternary_energy_equals_per_component_form():
    """Interior of the ternary bulk energy (Sec. 2.1, Eq. (3) under the
    constraint Eq. (1)): the C1 C2 C3 (Sigma_1 C1 + Sigma_2 C2 + Sigma_3 C3)
    and Lambda C1^2 C2^2 C3^2 terms are checked against the per-component
    form on states with all three components present, Lambda > 0."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        s, S, lam = _random_ternary(rng)
        p = params(s[0], s[1], s[2], lam)
        c = rng.dirichlet([1.5, 1.5, 1.5])
        c[2] = 1.0 - c[0] - c[1]
        ref = _energy_sum_form(S, lam, c)
        assert abs(pfo.bulk_energy(p, *c) - ref) <= 1e-14 * abs(ref) + 1e-20


def test_ternary_potential_from_per_component_energy():
    """Bulk chemical potentials (Sec. 2.1, Eq. (5) with lap C = 0):
    dE0/dC_i - dE0/dC_j is the derivative of E0 along e_i - e_j, a direction
    inside the plane C1 + C2 + C3 = 1, so it can be taken by central finite
    differences of the per-component form alone; then
    mu_i = (4 Sigma_T / xi) sum_{j != i} (that derivative) / Sigma_j with
    3 / Sigma_T = sum 1 / Sigma_i (Eq. (7))."""
    rng = np.random.default_rng(12)
    xi = 4.0
    for _ in range(100):
        s, S, lam = _random_ternary(rng)
        p = params(s[0], s[1], s[2], lam, xi)
        c = rng.dirichlet([2.0, 2.0, 2.0])
        ST = 3.0 / (1.0 / S).sum()
        h = 1e-5
        ref = np.zeros(3)
        for i in range(3):
            for j in range(3):
                if j == i:
                    continue
                e = np.zeros(3)
                e[i], e[j] = 1.0, -1.0
                dij = (_energy_sum_form(S, lam, c + h * e) - _energy_sum_form(S, lam, c - h * e)) / (2 * h)
                ref[i] += 4.0 * ST / xi * dij / S[j]
        mu = pfo.chem_potential(p, c, [0.0, 0.0, 0.0])
        scale = np.abs(ref).max()
        assert np.abs(mu - ref).max() < 1e-8 * scale, (mu, ref)


def test_ternary_gradient_term_per_component():
    """The gradient part of Eq. (5) is -(3/4) xi Sigma_i lap C_i for each
    component on its own: with the bulk part removed (a pure state, where
    E0 and all its derivatives vanish) mu_i carries only that term."""
    rng = np.random.default_rng(13)
    for _ in range(20):
        s, S, lam = _random_ternary(rng)
        xi = rng.uniform(3.0, 5.0)
        p = params(s[0], s[1], s[2], lam, xi)
        lap = rng.normal(0, 1e-2, 3)
        lap[2] = -lap[0] - lap[1]
        mu = pfo.chem_potential(p, [0.0, 0.0, 1.0], lap)
        assert np.abs(mu + 0.75 * xi * S * lap).max() < 1e-16
