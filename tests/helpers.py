"""Shared helpers of the test suite (comparison metrics)."""
import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def max_norms(m, o):
    """Pointwise errors of a GPU result m against the oracle's o: max |du|
    relative to max |u| of the oracle, and max |dC| (C is of order 1)."""
    du = np.abs(np.asarray(m["u"], np.float64) - o["u"]).max() / max(np.abs(o["u"]).max(), 1e-300)
    dc = float(np.abs(np.asarray(m["phi"], np.float64) - o["phi"]).max())
    return float(du), dc
