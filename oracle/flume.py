"""The flume study of Sec. 3.3.2 and the sensitivity measures of Sec. 3.4 (test
infrastructure only: the tests, and nothing on the product path, use this module).

normal_depth: the depth of uniform flow of discharge q per unit width down a bed of slope m
under the friction law of Appendix A (momentum sink K |v| v with K = alpha_p h (1 - theta) +
theta alpha_s, discharge q = theta h v): the gravity drive g theta h m balances K v^2.
hbar: eq. eq_h_bar, the mean steady depth over the cells of the vegetated zone x >= 9.
sensitivities: delta_s and delta_p of Sec. 3.4, the mean forward differences of hbar along
the alpha_s and the alpha_p axes of a regular grid.
"""
from __future__ import annotations

import numpy as np


def normal_depth(q, theta, m, alpha_s, alpha_p, g=9.81):
    def excess(h):  # drive minus friction; increasing in h
        v = q / (theta * h)
        K = alpha_p * h * (1.0 - theta) + theta * alpha_s
        return g * theta * h * m - K * v * v
    lo, hi = 1e-6, 1.0
    while excess(hi) < 0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if excess(mid) < 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def hbar(zone, h):
    """Mean depth over the cells of the zone (eq. eq_h_bar)."""
    zone = np.asarray(zone, bool)
    return float(np.asarray(h, np.float64)[zone].sum() / zone.sum())


def sensitivities(H, ds, dp):
    """delta_s, delta_p of Sec. 3.4 from H[i, j] = hbar at (alpha_s^i, alpha_p^j)."""
    H = np.asarray(H, np.float64)
    Ns, Np = H.shape
    d_s = 0.0
    for i in range(Ns - 1):
        for j in range(Np):
            d_s += (H[i + 1, j] - H[i, j]) / ds
    d_p = 0.0
    for i in range(Ns):
        for j in range(Np - 1):
            d_p += (H[i, j + 1] - H[i, j]) / dp
    return d_s / ((Ns - 1) * Np), d_p / (Ns * (Np - 1))
