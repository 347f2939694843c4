"""Parity on grids that are not squares or cubes, on the largest control
set, and on a problem without target nodes.

Square grids cannot tell the axes apart: an x / y swap in an index, a tile
count or a halo offset gives the same result when n[0] == n[1].  These
cases use a different node count, box length and tile remainder per axis.
Bars as in the other parity tests: labels and FP64 values bit-exact, FP32
within 1e-5 of the FP64 oracle."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available()
    from paper_1109_3577_amd import hjb
    return hjb


def _zeros(n, fp64):
    import torch
    return torch.empty(n, dtype=torch.float64 if fp64 else torch.float32, device="cuda")


def _np(t):
    return t.double().cpu().numpy()


def _box_problem(pr, dim, n, lo, hi, nc, R, fp32, drift=False, with_target=True):
    """Variable speed on a box with its own node count and length per axis;
    target ball off the centre split into R angular sectors (around z in
    3D); h is the smallest spacing, so the reach stays within one cell."""
    k = [(hi[d] - lo[d]) / (n[d] - 1) for d in range(dim)]
    h = min(k)
    X = pr.grid_coords(dim, n, lo, hi)
    c = 1.0 + 0.4 * np.sin(2.0 * math.pi * X[0] / (hi[0] - lo[0])) * np.cos(
        math.pi * X[1] / (hi[1] - lo[1]))
    w = None
    if drift:
        w = np.stack([0.2 * np.sin(math.pi * X[1])] + [0.2 * np.cos(math.pi * X[0])]
                     + ([0.1 * np.sin(math.pi * X[0])] if dim == 3 else []), axis=1)
    centre = [0.3 * lo[d] + 0.1 * hi[d] for d in range(dim)]
    r2 = sum((X[d] - centre[d]) ** 2 for d in range(dim))
    inside = (r2 <= 0.35 ** 2) if with_target else np.zeros(r2.shape, dtype=bool)
    ang = np.arctan2(X[1] - centre[1], X[0] - centre[0])
    part = np.floor((ang + math.pi) / (2.0 * math.pi) * R).astype(np.int64) % R
    tp = np.where(inside, part, -1).astype(np.int16)
    ctl = pr.unit_controls_2d(nc) if dim == 2 else pr.fibonacci_controls_3d(nc)
    return pr._make(dim, n, h, ctl, c, w, tp, R, fp32, f"box{dim}d", lo=lo, hi=hi)


def _pair(pr, dim, n, nc_grid, lo, hi, nc, R, drift=False, with_target=True):
    f = _box_problem(pr, dim, n, lo, hi, nc, R, True, drift, with_target)
    c = _box_problem(pr, dim, nc_grid, lo, hi, nc, R, False, drift, with_target)
    return f, c


def _check(H, orc, f, c):
    out = orc.patchy(f, c)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    assert np.array_equal(ph.u0(), out["u0"])
    assert np.array_equal(ph.feedback(), out["feedback"])
    assert np.array_equal(ph.labels(), out["labels"])
    v64 = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, v64)
    assert np.array_equal(_np(v64), out["v"])
    v32 = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, v32)
    assert np.abs(_np(v32) - out["v"]).max() <= 1e-5
    return out


@pytest.mark.parametrize("drift", [False, True])
def test_rectangular_2d(H, orc, pr, drift):
    """95 x 63 nodes on [-1.5, 1.5] x [-1, 1] (32 x 8 tiles leave 31 and 7
    nodes over), coarse 25 x 17, 6 parts."""
    f, c = _pair(pr, 2, (95, 63), (25, 17), (-1.5, -1.0), (1.5, 1.0), 24, 6, drift)
    _check(H, orc, f, c)


def test_box_3d(H, orc, pr):
    """21 x 29 x 17 nodes on [-1, 1] x [-1.4, 1.4] x [-0.8, 0.8], coarse
    9 x 13 x 9, 98 controls, 4 parts."""
    f, c = _pair(pr, 3, (21, 29, 17), (9, 13, 9), (-1.0, -1.4, -0.8), (1.0, 1.4, 0.8), 98, 4,
                 drift=True)
    _check(H, orc, f, c)


def test_largest_control_set(H, orc, pr):
    """N_c = 255 (the most the feedback byte holds) on a 41 x 37 grid."""
    f, c = _pair(pr, 2, (41, 37), (11, 10), (-1.0, -0.9), (1.0, 0.9), 255, 3)
    out = _check(H, orc, f, c)
    fb = out["feedback"]
    assert fb[f.target_part < 0].max() > 200 and np.all(fb[f.target_part >= 0] == 255)


def test_no_target_nodes(H, orc, pr):
    """No node lies in the target: no colour reaches any node, every label
    is -1 and the merged value is 1 everywhere (Kruzkov image of T = inf)."""
    f, c = _pair(pr, 2, (40, 33), (12, 10), (-1.0, -1.0), (1.0, 0.8), 16, 2, with_target=False)
    out = _check(H, orc, f, c)
    assert np.all(out["labels"] == -1) and np.all(out["v"] == 1.0)
