"""Writes the stored oracle results the GPU tests compare against.

Calls only the CPU oracle (oracle/) and the seeded problem generators; run
from the repository root:  python tests/golden/make_golden.py
Outputs (compressed numpy archives next to this script):
  config2_s0_full.npz   -- 1025^2 / 65^2, 16 parts, seed 0: coarse values,
                           feedback and labels of Steps 1-3.1.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1109_3577_amd import problems  # noqa: E402


def config2_full(seed=0):
    f, c = problems.config2(seed)
    t = time.time()
    vc, _ = O.solve_global(c)
    u0 = O.prolong(c, vc, f)
    fb = O.feedback(f, u0)
    lab = O.labels(f, fb)
    print(f"config2 seed {seed}: oracle Steps 1-3.1 in {time.time() - t:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, f"config2_s{seed}_full.npz"), v_coarse=vc,
                        feedback=fb, labels=lab)


if __name__ == "__main__":
    O.build(force=False)
    config2_full(0)
