"""Stress-concentration factors of the plate-with-hole scene, read off the
particles (test-side analysis, applied alike to the oracle's and the GPU
library's output).

sigma0 is the mean sigma_xx of the points more than 3 m from the hole's
centre along the load axis (x), where the strip is in uniform tension; the
factors are the largest sigma_xx / sigma0 over all points, and the smallest
sigma_xx / sigma0 and sigma_yy / sigma0 over the points within half a cell
of the hole's edge.  The paper's Table 1 lists, against Howland's
semi-analytical solution, the largest sigma_xx / sigma0 (3.13 against
3.14), the smallest (-0.029 against 0.00) and sigma_yy / sigma0 at the hole
(-1.08 against -1.11).
"""
import numpy as np

TABLE_1 = {"howland": {"max_sxx": 3.14, "min_sxx": 0.00, "min_syy": -1.11},
           "paper": {"max_sxx": 3.13, "min_sxx": -0.029, "min_syy": -1.08}}


def stress_concentration(x, sig, radius=0.5, h=0.0625, far_x=3.0):
    x = np.asarray(x, dtype=np.float64)
    sig = np.asarray(sig, dtype=np.float64)
    s0 = float(sig[x[:, 0] > far_x, 0].mean())
    ring = np.hypot(x[:, 0], x[:, 1]) < radius + h / 2
    return {"sigma0": s0, "max_sxx": float(sig[:, 0].max() / s0), "min_sxx": float(sig[ring, 0].min() / s0),
            "min_syy": float(sig[ring, 1].min() / s0)}
