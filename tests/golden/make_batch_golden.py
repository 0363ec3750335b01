"""Writes batch_large_500.npz: the oracle's state after 500 USF steps of the
four largest scenes of the batched set (256 independent elastic or
Drucker-Prager blocks, 1k-250k particles, 0.02 m cells, CFL 0.3).

Calls only the oracle and the seeded input generator.  For each of the four
scenes (by particle count) stores its index in the set, every 97th
particle's final position, velocity, stress and volume with its initial
position, and the particles-per-cell histogram of the final positions
(uint16).  Takes a few minutes on one core.

    python tests/golden/make_batch_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1909_13380_amd import scenes  # noqa: E402

STRIDE = 97
COUNT = 4


def main():
    scs = scenes.c3()
    order = np.argsort([len(sc["x"]) for sc in scs])[::-1][:COUNT]
    out = {"scenes": np.asarray(order, dtype=np.int64), "stride": STRIDE}
    t0 = time.time()
    for i in order:
        sc = scs[i]
        r = oracle.run(sc, sc["nsteps"])
        idx = np.arange(0, len(sc["x"]), STRIDE)
        out[f"s{i}_index"] = idx
        out[f"s{i}_nsteps"] = sc["nsteps"]
        out[f"s{i}_x0"] = sc["x"][idx]
        for k in ("x", "v", "stress", "vol"):
            out[f"s{i}_{k}"] = r[k][idx]
        out[f"s{i}_hist"] = oracle.cell_counts(sc["mesh"], r["x"]).astype(np.uint16)
        print(f"scene {i}: {len(sc['x'])} particles, {sc['nsteps']} steps, {time.time() - t0:.0f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_large_500.npz")
    np.savez_compressed(path, **out)
    print("wrote", path, os.path.getsize(path), "bytes")


if __name__ == "__main__":
    main()
