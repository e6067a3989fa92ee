"""Writes tests/golden/plummer16k_salpeter_one_step.txt: the oracle's state
after one global step (dt = 1/64, eta = 0.01, eps = 0) of the 16 384-body
Salpeter Plummer workload, at 512 sampled particles, with the step's
statistics.  Calls only the oracle and the input generator (about two minutes
on one core).  Run from the repository root:

    python tests/golden/make_plummer16k_step.py
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "plummer16k_salpeter_one_step.txt")
NSAMPLE = 512
SEED = 16384


def main():
    p = synth.workload(2)
    ref = p.copy()
    t0 = time.time()
    _, st = oracle.evolve(ref, 1 / 64, 1 / 64, oracle.Params(eta=0.01))
    t1 = time.time()
    idx = np.sort(np.random.default_rng(SEED).choice(p.n, NSAMPLE, replace=False))
    with open(OUT, "w") as f:
        f.write("# oracle: one CC global step (dt = 1/64, eta = 0.01, eps = 0) of synth.workload(2)\n")
        f.write(f"# (16384-body Plummer sphere, Salpeter 0.1-100), written by make_plummer16k_step.py "
                f"in {t1 - t0:.0f} s\n")
        f.write("# stats " + " ".join(f"{k}={v}" for k, v in st.items()) + "\n")
        f.write("# index x y z vx vy vz (float.hex)\n")
        for i in idx:
            f.write(str(int(i)) + " " + " ".join(float(getattr(ref, c)[i]).hex()
                                             for c in ("x", "y", "z", "vx", "vy", "vz")) + "\n")
    print(f"wrote {OUT} ({t1 - t0:.0f} s)")


if __name__ == "__main__":
    main()
