"""The learned preconditioner stage as a composition of linear-algebra steps.

TEST INFRASTRUCTURE ONLY (see the package header).  The network itself is not
part of the paper; the stage only decides how a network's prediction c enters
flexible GMRES next to the field-split preconditioner of Sec. 3 (eqs.
P_preconditioner / P_group):

    z0 = P_FS^{-1} v,  r1 = v - K z0,
    alpha = <r1, K c> / ||K c||^2   (0 when not finite or ||K c|| = 0),
    z = z0 + alpha c.

alpha is the least-squares step along c: it minimises ||v - K (z0 + alpha c)||,
so ||v - K z|| <= ||v - K z0||, with equality only when K c is orthogonal to r1.

Pins (tests/test_oracle_learned.py): the minimisation property against a scan
of alpha, the exact inverse when c is the exact error K^{-1} r1 (alpha = 1,
z = K^{-1} v), and the fallback alpha = 0 for a non-finite c.
"""
from __future__ import annotations

import numpy as np


def stage(apply_K, apply_fs, v: np.ndarray, c: np.ndarray):
    """Returns (z, alpha, r1) for one stage application with prediction c."""
    z0 = apply_fs(v)
    r1 = v - apply_K(z0)
    kc = apply_K(c)
    num = float(np.dot(r1, kc))
    den = float(np.dot(kc, kc))
    alpha = num / den if (np.isfinite(num) and np.isfinite(den) and den > 0.0) else 0.0
    z = z0 + alpha * c if alpha != 0.0 else z0.copy()
    return z, alpha, r1
