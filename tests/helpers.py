"""Error metrics shared by the parity tests."""

import numpy as np


def floored_rel(a, r, floor):
    """max |a - r| / max(|r|, floor) elementwise."""
    a = np.asarray(a).reshape(-1)
    r = np.asarray(r).reshape(-1)
    return float(np.max(np.abs(a - r) / np.maximum(np.abs(r), floor))) if r.size else 0.0


def l2_rel(a, r):
    a = np.asarray(a).reshape(-1)
    r = np.asarray(r).reshape(-1)
    nr = np.linalg.norm(r)
    return float(np.linalg.norm(a - r) / nr) if nr > 0 else float(np.linalg.norm(a))
