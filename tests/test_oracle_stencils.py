"""Pins of the oracle's finite-difference stencils: exactness on polynomials
(closed forms) and the wall/periodic ghost handling against an explicitly
padded array (brute force with numpy's symmetric and wrap padding)."""
import numpy as np
import pytest

from oracle import pfo

NX, NY = 12, 11


def poly_field(cx, cy, cxx, cyy, cxy):
    y, x = np.meshgrid(np.arange(NY, dtype=float), np.arange(NX, dtype=float), indexing="ij")
    f = 0.3 + cx * x + cy * y + cxx * x * x + cyy * y * y + cxy * x * y
    gx = cx + 2 * cxx * x + cxy * y
    gy = cy + 2 * cyy * y + cxy * x
    lap = 2 * cxx + 2 * cyy
    return f, gx, gy, lap


INTERIOR = (slice(2, NY - 2), slice(2, NX - 2))


@pytest.mark.parametrize("coef", [(0.1, -0.2, 0.0, 0.0, 0.0), (0.05, 0.02, 0.01, -0.03, 0.02)])
def test_central_gradient_and_laplacian_exact_on_quadratics(coef):
    f, gx, gy, lap = poly_field(*coef)
    g = pfo.stencil(f, "grad_cd")
    l = pfo.stencil(f, "lap_cd")
    assert np.allclose(g[0][INTERIOR], gx[INTERIOR], atol=1e-12)
    assert np.allclose(g[1][INTERIOR], gy[INTERIOR], atol=1e-12)
    assert np.allclose(l[INTERIOR], lap, atol=1e-12)


def test_mixed_directional_derivative_exact_on_quadratics():
    ex, ey, w, opp = pfo.lattice()
    f, gx, gy, lap = poly_field(0.05, 0.02, 0.01, -0.03, 0.02)
    for a in range(1, 9):
        d = pfo.stencil(f, "dir_md", a)
        exact = ex[a] * gx + ey[a] * gy
        assert np.allclose(d[INTERIOR], exact[INTERIOR], atol=1e-12), a


def test_mixed_gradient_exact_on_quadratics():
    f, gx, gy, lap = poly_field(0.05, 0.02, 0.01, -0.03, 0.02)
    g = pfo.stencil(f, "grad_md")
    assert np.allclose(g[0][INTERIOR], gx[INTERIOR], atol=1e-12)
    assert np.allclose(g[1][INTERIOR], gy[INTERIOR], atol=1e-12)


def test_md_differs_from_cd_on_cubics():
    # the mixed derivative is the mean of the central and the biased forms:
    # on a cubic it carries -(e.grad)^3 f / 12 where the central one carries +(e.grad)^3 f / 6
    y, x = np.meshgrid(np.arange(NY, dtype=float), np.arange(NX, dtype=float), indexing="ij")
    f = 0.001 * x ** 3
    d_md = pfo.stencil(f, "dir_md", 1)
    d_cd = pfo.stencil(f, "dir_cd", 1)
    exact = 0.003 * x ** 2
    assert np.allclose((d_md - exact)[INTERIOR], -0.001 * 6 / 12, atol=1e-12)
    assert np.allclose((d_cd - exact)[INTERIOR], 0.001 * 6 / 6, atol=1e-12)


def padded_reference(f, kind, a=0):
    """Brute force: pad with the wall mirror (numpy 'symmetric') in y and the
    period ('wrap') in x, then apply the textbook stencil with plain loops."""
    ex, ey, w, opp = pfo.lattice()
    P = np.pad(np.pad(f, ((2, 2), (0, 0)), mode="symmetric"), ((0, 0), (2, 2)), mode="wrap")
    out = np.zeros((2,) + f.shape) if kind.startswith("grad") else np.zeros(f.shape)
    cs2 = 1.0 / 3.0
    for y in range(f.shape[0]):
        for x in range(f.shape[1]):
            F = lambda dx, dy: P[y + 2 + dy, x + 2 + dx]
            if kind == "grad_cd":
                for b in range(1, 9):
                    out[0, y, x] += w[b] * ex[b] * (F(ex[b], ey[b]) - F(-ex[b], -ey[b])) / (2 * cs2)
                    out[1, y, x] += w[b] * ey[b] * (F(ex[b], ey[b]) - F(-ex[b], -ey[b])) / (2 * cs2)
            elif kind == "lap_cd":
                for b in range(1, 9):
                    out[y, x] += w[b] * (F(ex[b], ey[b]) - 2 * F(0, 0) + F(-ex[b], -ey[b])) / cs2
            elif kind == "dir_md":
                out[y, x] = (-F(2 * ex[a], 2 * ey[a]) + 5 * F(ex[a], ey[a]) - 3 * F(0, 0) - F(-ex[a], -ey[a])) / 4
    return out


@pytest.mark.parametrize("kind,a", [("grad_cd", 0), ("lap_cd", 0), ("dir_md", 2), ("dir_md", 7), ("dir_md", 5)])
def test_boundary_ghosts_match_padding(kind, a):
    rng = np.random.default_rng(3)
    f = rng.standard_normal((NY, NX))
    got = pfo.stencil(f, kind, a)
    ref = padded_reference(f, kind, a)
    assert np.allclose(got, ref, atol=1e-13)
