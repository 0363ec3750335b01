"""Writes c5sub_<shape>_500.npz: the oracle's state after all 500 steps of
the 1/64 subsample of the large GIMP column (Drucker-Prager block of
64x32x24 cells, 393,216 particles, 128x64x32 mesh of 0.005 m cells,
dt = 1e-5 s), with GIMP or linear shape functions.

Calls only the oracle and the seeded input generator.  Stores every 64th
particle's final position, velocity, stress and volume, and the cell
histograms (uint8) of the final and initial positions.

    python tests/golden/make_c5sub_golden.py gimp|linear [nsteps]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1909_13380_amd import scenes  # noqa: E402

STRIDE = 64


def main(shape_name: str, nsteps: int = 500):
    shape = {"gimp": scenes.SHAPE_GIMP, "linear": scenes.SHAPE_LINEAR}[shape_name]
    sc = scenes.c5(subsample=True, shape=shape)
    grid = oracle.Grid(sc["mesh"], shape)
    state = {k: sc[k] for k in ("x", "v", "stress", "vol", "mass")}
    hist0 = oracle.cell_counts(sc["mesh"], sc["x"])
    t0 = time.time()
    done = 0
    while done < nsteps:
        k = min(25, nsteps - done)
        state = oracle.run(sc, k, grid=grid, state=state)
        done += k
        print(f"step {done}/{nsteps}  {time.time() - t0:.0f} s", flush=True)
    hist = oracle.cell_counts(sc["mesh"], state["x"])
    idx = np.arange(0, len(sc["x"]), STRIDE)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"c5sub_{shape_name}_{nsteps}.npz")
    np.savez_compressed(out, index=idx, nsteps=nsteps, x0=sc["x"][idx], x=state["x"][idx], v=state["v"][idx],
                        stress=state["stress"][idx], vol=state["vol"][idx],
                        hist=hist.astype(np.uint8), hist0=hist0.astype(np.uint8))
    print("wrote", out, os.path.getsize(out), "bytes")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 500)
