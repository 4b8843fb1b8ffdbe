"""Write c4_smallest_energy.txt: total energy E = sum 1/2 m v^2 + sum m u of
the smallest served-integration request (blob-in-lattice, 23^3 particles,
seed 4051) over 200 kick-drift-kick steps with the global Courant step,
computed by the brute-force oracle only.

    python tests/golden/make_c4_energy.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1709_04488_amd import workloads as W  # noqa: E402

SIDE, SEED, STEPS = 23, 4051, 200


def main():
    oracle.build(force=False)
    w = W.blob_in_lattice(SIDE, seed=SEED)
    a = w.arrays
    t0 = time.time()
    _, energy, dts = oracle.kdk(oracle.Params(**w.setup), a["x"], a["y"], a["z"], a["vx"], a["vy"],
                                a["vz"], a["m"], a["u"], a["h"], STEPS, 0.0)
    el = time.time() - t0
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_smallest_energy.txt")
    with open(out, "w") as f:
        f.write(f"# oracle KDK, blob_in_lattice({SIDE}, seed={SEED}), N={w.n}, {STEPS} steps, "
                f"global Courant step (C=0.2), FP64 brute force\n")
        f.write(f"# written by tests/golden/make_c4_energy.py in {el:.0f} s on "
                f"{oracle.num_threads()} threads\n")
        f.write("# step  time  E\n")
        t = 0.0
        for k in range(STEPS + 1):
            f.write(f"{k} {t:.17g} {energy[k]:.17g}\n")
            if k < STEPS:
                t += dts[k]
    print(out, el, (energy[-1] - energy[0]) / energy[0])


if __name__ == "__main__":
    main()
