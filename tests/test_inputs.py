"""Host-side input generators: SplitMix64 against its published reference
values, and the boxed evaluation of the bubble profile against the direct
formula evaluated on every node."""
import numpy as np

from paper_2207_09431_amd import inputs


def test_splitmix64_reference_values():
    # first outputs of SplitMix64 seeded with 1234567 (Vigna's reference C
    # implementation, splitmix64.c)
    ref = [6457827717110365317, 3203168211198807973, 9817491932198370423,
           4593380528125082431, 16408922859458223821]
    assert [int(v) for v in inputs.splitmix64(1234567, 5)] == ref


def test_uniform_range_and_slices():
    u = inputs.uniform(3, 1000, -2.0, 5.0)
    assert u.min() >= -2.0 and u.max() < 5.0
    assert np.array_equal(inputs.uniform(3, 10, offset=990), inputs.uniform(3, 1000)[990:])


def _direct(nx, ny, bubbles, xi):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    c = np.zeros((ny, nx))
    for (cx, cy, r) in bubbles:
        dx = x - cx
        dx = dx - nx * np.round(dx / nx)
        c += 0.5 - 0.5 * np.tanh((np.sqrt(dx * dx + (y - cy) ** 2) - r) / (0.5 * xi))
    return np.minimum(c, 1.0)


def test_bubble_field_box_equals_direct_formula():
    cases = [(300, 600, inputs.place_bubbles(300, 600, 3, 25.0, 40.0, 4.0, 9)),
             (64, 128, [(32.0, 32.0, 8.0)]),
             (200, 400, [(1.5, 120.0, 25.0)]),          # straddles the periodic seam
             (100, 100, [(50.0, 50.0, 45.0)]),         # box wider than the domain
             (120, 90, [(60.0, 2.0, 10.0), (118.0, 85.0, 12.0)])]
    for nx, ny, b in cases:
        assert np.array_equal(inputs.bubble_field(nx, ny, b, 4.0), _direct(nx, ny, b, 4.0))


def test_place_bubbles_constraints():
    b = inputs.place_bubbles(512, 1024, 12, 25.0, 40.0, 4.0, 5)
    for i, (x, y, r) in enumerate(b):
        assert 25.0 <= r < 40.0 and y - r >= 8.0 and y + r <= 1024 - 8.0
        for (x2, y2, r2) in b[:i]:
            dx = (x - x2) - 512 * round((x - x2) / 512)
            assert dx * dx + (y - y2) ** 2 >= (r + r2 + 8.0) ** 2


def test_rest_pressure_hydrostatic_and_laplace():
    nx, ny, xi, sigma, rho_l, g = 200, 300, 4.0, 1e-4, 1.0, 2e-7
    bubbles = [(60.0, 100.0, 25.0), (150.0, 220.0, 30.0)]
    p = inputs.rest_pressure(nx, ny, bubbles, xi, sigma, rho_l, g)
    yc = 0.5 * (ny - 1)
    # far from every bubble: the liquid's hydrostatic profile, exactly
    for (x, y) in [(5, 10), (190, 20), (110, 150), (20, 290)]:
        assert p[y, x] == rho_l * g * (yc - y)
    # at a centre: the liquid pressure at that height plus sigma / R
    for (cx, cy, r) in bubbles:
        want = rho_l * g * (yc - cy) + sigma / r
        assert abs(p[int(cy), int(cx)] - want) < 1e-6 * sigma / r
    # inside a bubble the pressure carries no hydrostatic gradient
    cx, cy, r = bubbles[0]
    assert abs(p[int(cy) + 10, int(cx)] - p[int(cy) - 10, int(cx)]) < 1e-4 * sigma / r
