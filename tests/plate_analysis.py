"""Stress-concentration factors of the plate-with-hole scene, read off the
particles (test-side analysis, applied alike to the oracle's and the GPU
library's output).

Reading of the paper's Table 1 (benchmark section), whose three rows are:
  - "maximum sigma_xx / sigma0" (Howland 3.14, the paper's MPM 3.13): the
    largest sigma_xx / sigma0 over all points; it sits at the hole's edge on
    the axis across the load, (0, a);
  - "minimum sigma_xx / sigma0" (0.00, -0.029) and "maximum sigma_yy /
    sigma0" (-1.11, -1.08): sigma_xx and sigma_yy at the hole's edge on the
    load axis, (a, 0), where the free edge makes sigma_xx vanish exactly and
    the hoop stress sigma_yy is the most compressive.  Howland's 0.00 is that
    free-edge value: the edge's smallest sigma_xx over all angles is about
    -sigma0/16 (at 21 degrees, infinite-plate solution), not zero.
The value at a point is that of the particle nearest to it.  sigma0 is the
applied end traction, 100 Pa.
"""
import numpy as np

TABLE_1 = {"howland": {"max_sxx": 3.14, "min_sxx": 0.00, "max_syy": -1.11},
           "paper": {"max_sxx": 3.13, "min_sxx": -0.029, "max_syy": -1.08}}


def stress_concentration(x, sig, radius=0.5, sigma0=100.0, far_x=3.0):
    x = np.asarray(x, dtype=np.float64)
    sig = np.asarray(sig, dtype=np.float64)
    edge = int(np.argmin(np.hypot(x[:, 0] - radius, x[:, 1])))   # nearest to (a, 0)
    return {"far_sxx": float(sig[x[:, 0] > far_x, 0].mean() / sigma0),
            "max_sxx": float(sig[:, 0].max() / sigma0),
            "min_sxx": float(sig[edge, 0] / sigma0),
            "max_syy": float(sig[edge, 1] / sigma0)}
