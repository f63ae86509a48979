"""Pins of the oracle's D2Q9 tables against textbook lattice identities
(Sec. 2.2, Eqs. (10)-(11)): weights sum to one, odd moments vanish, the second
moment is c_s^2 I with c_s^2 = 1/3, the fourth moment is isotropic."""
import numpy as np

from oracle import pfo


def test_lattice_moments():
    ex, ey, w, opp = pfo.lattice()
    e = np.stack([ex, ey], axis=1).astype(float)
    cs2 = 1.0 / 3.0
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose((w[:, None] * e).sum(0), 0.0, atol=1e-15)
    M2 = np.einsum("a,ai,aj->ij", w, e, e)
    assert np.allclose(M2, cs2 * np.eye(2), atol=1e-15)
    M3 = np.einsum("a,ai,aj,ak->ijk", w, e, e, e)
    assert np.allclose(M3, 0.0, atol=1e-15)
    M4 = np.einsum("a,ai,aj,ak,al->ijkl", w, e, e, e, e)
    d = np.eye(2)
    iso = cs2 * cs2 * (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d))
    assert np.allclose(M4, iso, atol=1e-15)


def test_lattice_order_and_opposites():
    ex, ey, w, opp = pfo.lattice()
    # alpha = 0 rest, 1-4 along cos/sin((alpha-1) pi/2), 5-8 diagonals at (2 alpha - 9) pi / 4
    for a in range(1, 5):
        t = (a - 1) * np.pi / 2
        assert (ex[a], ey[a]) == (round(np.cos(t)), round(np.sin(t)))
        assert w[a] == 1.0 / 9.0
    for a in range(5, 9):
        t = (2 * a - 9) * np.pi / 4
        assert (ex[a], ey[a]) == (round(np.sqrt(2) * np.cos(t)), round(np.sqrt(2) * np.sin(t)))
        assert w[a] == 1.0 / 36.0
    assert w[0] == 4.0 / 9.0
    for a in range(9):
        assert ex[opp[a]] == -ex[a] and ey[opp[a]] == -ey[a]
