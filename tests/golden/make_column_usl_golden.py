"""Writes column_2m_usl_200.npz: the oracle's state after 200 update-stress-
last (USL) steps of the granular column (Drucker-Prager block of 64x32x128
cells, 2,097,152 particles, 256x128x160 mesh of 0.01 m cells, dt = 2e-5 s);
with the argument musl, column_2m_musl_200.npz from 200 modified-USL steps.

Calls only the oracle and the seeded input generator.  Stores every 1024th
particle's final position, velocity, stress and volume, plus the cell
histogram of the final positions (uint8) and of the initial ones.  Takes a
few minutes on one core.

    python tests/golden/make_column_usl_golden.py [nsteps] [usl|musl]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1909_13380_amd import scenes  # noqa: E402

STRIDE = 1024


def main(nsteps: int = 200, algo: str = "usl"):
    sc = scenes.c2()
    sc["scheme"]["algo"] = {"usl": scenes.USL, "musl": scenes.MUSL}[algo]
    grid = oracle.Grid(sc["mesh"], oracle.SHAPE_LINEAR)
    state = {k: sc[k] for k in ("x", "v", "stress", "vol", "mass")}
    hist0 = oracle.cell_counts(sc["mesh"], sc["x"])
    t0 = time.time()
    done = 0
    while done < nsteps:
        k = min(50, nsteps - done)
        state = oracle.run(sc, k, grid=grid, state=state)
        done += k
        print(f"step {done}/{nsteps}  {time.time() - t0:.0f} s", flush=True)
    hist = oracle.cell_counts(sc["mesh"], state["x"])
    idx = np.arange(0, len(sc["x"]), STRIDE)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"column_2m_{algo}_{nsteps}.npz")
    np.savez_compressed(out, index=idx, nsteps=nsteps, x0=sc["x"][idx], x=state["x"][idx], v=state["v"][idx],
                        stress=state["stress"][idx], vol=state["vol"][idx],
                        hist=hist.astype(np.uint8), hist0=hist0.astype(np.uint8))
    print("wrote", out, os.path.getsize(out), "bytes")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 200, sys.argv[2] if len(sys.argv) > 2 else "usl")
