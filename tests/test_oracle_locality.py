"""The dependency radius of one step is 3 nodes, and the macroscopic fields
add 1: the oracle's u, p, C on a region after k steps are the same, bit for
bit, whether the window around it extends 3k + 1 or more nodes beyond it, and
differ with a margin of 3k.  The full-size GPU parity test relies on this to
check sampled windows of the 2048 x 4096 domain."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from paper_2207_09431_amd import inputs  # noqa: E402
import test_gpu_fullsize as F  # noqa: E402


def test_windows_with_margin_3k_plus_1_are_exact():
    case = inputs.many_bubbles(512, 1024, 8, seed=5)
    case["u"] = inputs.velocity_noise(512, 1024, 11, 1e-4)
    steps = 4
    b = case["bubbles"][0]
    for (x0, y0) in [(int(b[0] + b[2]) - 32, int(b[1]) - 32), (40, 0), (512 - 32, 1024 - 64)]:
        a = F.oracle_window(case, x0 % 512, y0, steps, margin=3 * steps + 1)
        c = F.oracle_window(case, x0 % 512, y0, steps, margin=3 * steps + 9)
        for k in ("u", "phi", "p"):
            assert np.array_equal(a[k], c[k]), (x0, y0, k)


def test_margin_3k_is_not_exact():
    """A margin of 3k lets the window's own edges reach the region."""
    case = inputs.many_bubbles(512, 1024, 8, seed=5)
    case["u"] = inputs.velocity_noise(512, 1024, 11, 1e-4)
    steps = 3
    b = case["bubbles"][0]
    x0, y0 = int(b[0] + b[2]) - 32, int(b[1]) - 32
    a = F.oracle_window(case, x0, y0, steps, margin=3 * steps)
    c = F.oracle_window(case, x0, y0, steps, margin=3 * steps + 9)
    assert not np.array_equal(a["u"], c["u"])
