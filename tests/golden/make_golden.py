"""Writes the stored oracle results the GPU tests compare against.

Calls only the CPU oracle (oracle/) and the seeded problem generators; run
from the repository root:  python tests/golden/make_golden.py [names...]
Outputs (compressed numpy archives next to this script):
  config2_s0_full.npz   -- 2D variable speed 1025^2 / 65^2, 32 controls, 16
                           parts, seed 0: coarse values, feedback and labels
                           of Steps 1-3.1, and the merged patchy values of
                           Steps 3.2-4 (exact fixed point).
  config2_s0_513.npz    -- the same generator at 513^2 / 33^2: labels and
                           merged patchy values.
  config3_s0_65.npz     -- 3D variable speed 65^3 / 9^3, 98 controls, 64
                           parts, seed 0: labels and merged patchy values.
  config3_s0_129.npz    -- the same at 129^3 / 17^3: labels, and the merged
                           patchy values at 60,000 sampled nodes.
  config3_s0_257.npz    -- the same at the full 257^3 / 33^3: all labels, and
                           the merged patchy values at 100,000 sampled nodes
                           (a few hours of oracle time on 8 cores).
  config2_s0_1025_reading.npz -- the paper's own Step 3.1 transport (no
                           factor; scheme step, and the step |h_i f| = k) at
                           1025^2: part of the largest colour per node and
                           its band (>= 0.55, [0.5, 0.55), < 0.5).
Merged values are stored rounded to FP32 (`v32`, within 6e-8 of the FP64
oracle, far below the 1e-5 FP32 tolerance) next to the SHA-256 of the
oracle's FP64 bytes (`v64_sha256`), which an FP64 GPU result must match bit
for bit.
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1109_3577_amd import problems  # noqa: E402


def sha64(v) -> str:
    return hashlib.sha256(np.ascontiguousarray(v, dtype=np.float64).tobytes()).hexdigest()


def _patchy(f, c, what):
    t = time.time()
    r = O.patchy(f, c)
    lab, un, de = O.labels(f, r["feedback"], want_unreached=True, want_detached=True)
    assert np.array_equal(lab, r["labels"])
    print(f"{what}: oracle Steps 1-4 in {time.time() - t:.1f} s "
          f"(unreached {un}, detached {de})", flush=True)
    return r, de


def config2_full(seed=0):
    f, c = problems.config2(seed)
    r, de = _patchy(f, c, f"config2 seed {seed} 1025^2")
    np.savez_compressed(os.path.join(HERE, f"config2_s{seed}_full.npz"), v_coarse=r["v_coarse"],
                        feedback=r["feedback"], labels=r["labels"],
                        v32=r["v"].astype(np.float32), v64_sha256=sha64(r["v"]),
                        detached=np.int64(de))


def config2_side(n, seed=0):
    f, c = problems.config2(seed, n, problems.coarse_size_2d(n))
    r, de = _patchy(f, c, f"config2 seed {seed} {n}^2")
    np.savez_compressed(os.path.join(HERE, f"config2_s{seed}_{n}.npz"), labels=r["labels"],
                        v32=r["v"].astype(np.float32), v64_sha256=sha64(r["v"]),
                        detached=np.int64(de))


def coarse_size_3d(n):
    return min(33, max(9, round((n - 1) / 8) + 1))


def config3_side(n, seed=0, sample=None):
    f, c = problems.config3(seed, n, coarse_size_3d(n))
    r, de = _patchy(f, c, f"config3 seed {seed} {n}^3")
    out = dict(labels=r["labels"], v64_sha256=sha64(r["v"]), detached=np.int64(de))
    if sample is None:
        out["v32"] = r["v"].astype(np.float32)
    else:
        idx = np.sort(np.random.default_rng(129).choice(f.N, size=sample, replace=False))
        out["idx"] = idx.astype(np.int64)
        out["v64_at_idx"] = r["v"][idx]
    np.savez_compressed(os.path.join(HERE, f"config3_s{seed}_{n}.npz"), **out)


def config2_reading(seed=0, n=1025):
    """The paper's own colour transport at the full 2D size: eq.
    HJBridotta_discreta without the factor beta, with the scheme's step
    (plain) and with the step |h_i f| = k (paper); per node the part of the
    largest colour and whether that colour is >= 0.55, in [0.5, 0.55) or
    below 0.5 (2, 1, 0)."""
    f, c = problems.config2(seed, n, problems.coarse_size_2d(n))
    vc, _ = O.solve_global(c)
    fb = O.feedback(f, O.prolong(c, vc, f))
    out = {}
    for name, mode in (("plain", O.TRACE_PLAIN), ("paper", O.TRACE_PAPER)):
        t = time.time()
        best = np.zeros(f.N)
        arg = np.full(f.N, -1, dtype=np.int8)
        total = np.zeros(f.N)
        for j in range(f.n_parts):
            phi, sw, _ = O.trace_part_mode(f, fb, j, mode, max_sweeps=200000)
            up = phi > best
            best[up] = phi[up]
            arg[up] = j
            total += phi
        band = np.where(best >= 0.55, 2, np.where(best >= 0.5, 1, 0)).astype(np.uint8)
        out[f"{name}_part"] = arg
        out[f"{name}_band"] = band
        out[f"{name}_sum_dev"] = np.float64(np.abs(total[best > 0] - 1.0).max())
        print(f"reading {name} {n}^2: {time.time() - t:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, f"config2_s{seed}_{n}_reading.npz"), **out)


JOBS = {
    "config2_full": lambda: config2_full(0),
    "config2_513": lambda: config2_side(513),
    "config3_65": lambda: config3_side(65),
    "config3_129": lambda: config3_side(129, sample=60000),
    "config3_full": lambda: config3_side(257, sample=100000),
    "config2_reading": lambda: config2_reading(0),
}

if __name__ == "__main__":
    O.build(force=False)
    for name in (sys.argv[1:] or list(JOBS)):
        JOBS[name]()
