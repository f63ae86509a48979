"""The largest domain the boundary accepts: 16384 x 32767 nodes (pitch x ny
just below 2^29, so the float64 planes end within 0.03 % of the 2^32 bytes
that the kernels' 32-bit byte offsets address).  After 6 steps, three 64 x 64
windows are compared element by element with the oracle run on the window
plus a 3k + 2 margin: one at the far corner (top wall, right edge: the
largest offsets), one across the periodic seam near the top, one near the
origin."""
import numpy as np
import pytest

from oracle.pfo import Oracle
from paper_2207_09431_amd import inputs
from helpers import rel_l2

pytestmark = pytest.mark.gpu
NX, NY, K, WIN = 16384, 32767, 6, 64
MARGIN = 3 * K + 2


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("no GPU visible")
    return t


def oracle_window(prm, C, x0, y0):
    ya, yb = max(0, y0 - MARGIN), min(NY, y0 + WIN + MARGIN)
    xs = np.arange(x0 - MARGIN, x0 + WIN + MARGIN) % NX
    o = Oracle(dict(prm, nx=len(xs), ny=yb - ya))
    o.init_fields(np.ascontiguousarray(C[:, ya:yb][:, :, xs]))
    o.step(K)
    m = o.macroscopic()
    sl = (slice(y0 - ya, y0 - ya + WIN), slice(MARGIN, MARGIN + WIN))
    return m["u"][(slice(None),) + sl], m["phi"][(slice(None),) + sl]


def test_largest_domain_windows(torch):
    from paper_2207_09431_amd.pflbm import Solver
    prm = inputs.large_domain_params(NX, NY)
    bubbles = [(NX - 70.0, NY - 90.0, 30.0), (10.0, NY - 300.0, 30.0), (200.0, 150.0, 30.0)]
    C = inputs.bubble_field(NX, NY, bubbles, prm["xi"])[None]
    s = Solver(prm)
    s.set_variant(0)
    s.init_fields(0, C)
    s.step(K)
    m = s.macroscopic(0)
    s.synchronize()
    for (x0, y0) in [(NX - WIN, NY - WIN), (NX - WIN // 2, NY - 300 - WIN // 2), (170, 120)]:
        xs = torch.tensor(np.arange(x0, x0 + WIN) % NX, device=m["u"].device)
        gu = m["u"][:, y0:y0 + WIN][:, :, xs].double().cpu().numpy()
        gc = m["phi"][:, y0:y0 + WIN][:, :, xs].double().cpu().numpy()
        ou, oc = oracle_window(prm, C, x0, y0)
        ru, rc = rel_l2(gu, ou), rel_l2(gc, oc)
        print(f"window ({x0},{y0}) rel-L2 u {ru:.2e} C {rc:.2e}", flush=True)
        assert ru <= 1e-5 and rc <= 1e-5
    s.close()
