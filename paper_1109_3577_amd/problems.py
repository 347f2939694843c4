"""Seeded synthetic minimum-time problems (inputs only).

This module tabulates control problems of the family ``f(x, a) = c(x) a + w(x)``
on a uniform box grid and emits the arrays both the GPU library and the CPU
oracle consume.  It contains none of the scheme's arithmetic (no foot points,
no interpolation, no value iteration): only the problem statement of the
paper's eq. (HJB) in Section 1 -- box, target, dynamics and control set -- plus
the discretisation parameters h, k and beta = exp(-h) of Section 2.1.

Conventions shared by every consumer:

* nodes ``p = (p_x, p_y, p_z)``, flat index ``p_x + n_x (p_y + n_y p_z)``
  (x fastest); in 2D ``n_z = 1``;
* ``x_i = lo + i k`` with ``k = (hi - lo) / (n - 1)``;
* ``step[d] = h / k_d``: foot-point displacement in cells per unit of f;
* ``target_part[p] = -1`` for non-target nodes, else the index ``j`` of the
  part of the target the node belongs to (Section 3: the target is divided
  into R parts);
* ``beta = exp(-h)`` is computed here with the host libm; when the value grid
  is to be stored in FP32 the instance carries ``float32(exp(-h))`` so that
  beta and ``1 - beta`` are exact in both precisions; ``omb = 1 - beta`` is
  exact in FP64 because beta lies in [0.5, 1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Problem", "grid_coords", "unit_controls_2d", "fibonacci_controls_3d",
    "eikonal_2d", "config1", "variable_speed_2d", "config2", "config3",
    "variable_speed_3d", "line_target_2d", "zermelo_2d", "batched_problem",
    "config4", "ServingRequest", "serving_stream", "coarse_size_2d",
]


@dataclasses.dataclass
class Problem:
    """One tabulated minimum-time problem on a uniform grid."""

    dim: int
    n: tuple                   # (nx, ny, nz); nz == 1 in 2D
    lo: tuple
    hi: tuple
    h: float                   # fictitious time step
    step: tuple                # h / k_d per axis
    beta: float
    omb: float                 # 1 - beta, exact
    controls: np.ndarray       # float64 [Nc, dim]
    speed: np.ndarray          # float64 [N]
    drift: Optional[np.ndarray]  # float64 [N, dim] or None
    target_part: np.ndarray    # int16 [N]
    n_parts: int
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)
    # variable step of Section 2.1 (h_i with |h_i f| = k): per-node
    # beta_i = exp(-h_i), or None for the scalar beta
    beta_node: Optional[np.ndarray] = None
    # tabulated dynamics, control-major: foot-point displacement in cells
    # [Nc, N, dim] and beta per control and node [Nc, N] (either may be None)
    foot: Optional[np.ndarray] = None
    beta_pk: Optional[np.ndarray] = None

    @property
    def N(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def n_controls(self) -> int:
        return int(self.controls.shape[0])

    @property
    def shape(self) -> tuple:
        """numpy shape of a node array, slowest axis first."""
        if self.dim == 2:
            return (self.n[1], self.n[0])
        return (self.n[2], self.n[1], self.n[0])

    @property
    def k(self) -> tuple:
        return tuple((self.hi[d] - self.lo[d]) / (self.n[d] - 1) if self.n[d] > 1 else 0.0
                     for d in range(3))

    def coords(self) -> List[np.ndarray]:
        return grid_coords(self.dim, self.n, self.lo, self.hi)

    def is_target(self) -> np.ndarray:
        return self.target_part >= 0

    def validate(self) -> None:
        assert self.dim in (2, 3)
        assert self.controls.dtype == np.float64 and self.controls.shape[1] == self.dim
        assert self.speed.dtype == np.float64 and self.speed.shape == (self.N,)
        assert self.target_part.dtype == np.int16 and self.target_part.shape == (self.N,)
        if self.drift is not None:
            assert self.drift.dtype == np.float64 and self.drift.shape == (self.N, self.dim)
        assert 0.5 <= self.beta < 1.0 and self.omb == 1.0 - self.beta
        if self.beta_node is not None:
            assert self.beta_node.dtype == np.float64 and self.beta_node.shape == (self.N,)
            assert np.all((self.beta_node >= 0.0) & (self.beta_node < 1.0))


def grid_coords(dim: int, n: Sequence[int], lo: Sequence[float], hi: Sequence[float]):
    """Node coordinates, each flattened to length N in x-fastest order."""
    axes = []
    for d in range(dim):
        k = (hi[d] - lo[d]) / (n[d] - 1)
        axes.append(lo[d] + k * np.arange(n[d], dtype=np.float64))
    if dim == 2:
        Y, X = np.meshgrid(axes[1], axes[0], indexing="ij")
        return [X.ravel(), Y.ravel()]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return [X.ravel(), Y.ravel(), Z.ravel()]


def _snap(a: np.ndarray) -> np.ndarray:
    """Set components within 1e-15 of 0 or +-1 to that value exactly."""
    a = a.copy()
    for t in (0.0, 1.0, -1.0):
        a[np.abs(a - t) < 1e-15] = t
    return a


def unit_controls_2d(nc: int) -> np.ndarray:
    """N_c unit directions at angles 2 pi k / N_c (discretisation of B(0,1)
    boundary, Section 2.1: the minimum over A is taken over N_c points)."""
    th = 2.0 * math.pi * np.arange(nc) / nc
    return _snap(np.stack([np.cos(th), np.sin(th)], axis=1))


def fibonacci_controls_3d(nc: int = 98) -> np.ndarray:
    """N_c quasi-uniform unit vectors on S^2 (Fibonacci lattice)."""
    i = np.arange(nc, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / nc
    ph = i * math.pi * (3.0 - math.sqrt(5.0))
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return _snap(np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1))


def _beta(h: float, fp32: bool) -> float:
    b = math.exp(-h)
    if fp32:
        b = float(np.float32(b))
    return b


def _make(dim, n, h, controls, speed, drift, target_part, n_parts, fp32, name,
          lo=None, hi=None, meta=None) -> Problem:
    lo = tuple(lo if lo is not None else [-1.0] * dim) + (0.0,) * (3 - dim)
    hi = tuple(hi if hi is not None else [1.0] * dim) + (0.0,) * (3 - dim)
    nn = tuple(n) + (1,) * (3 - dim)
    k = [(hi[d] - lo[d]) / (nn[d] - 1) for d in range(dim)]
    step = tuple(h / k[d] for d in range(dim)) + (0.0,) * (3 - dim)
    b = _beta(h, fp32)
    p = Problem(dim=dim, n=nn, lo=lo, hi=hi, h=h, step=step, beta=b, omb=1.0 - b,
                controls=np.ascontiguousarray(controls, dtype=np.float64),
                speed=np.ascontiguousarray(speed, dtype=np.float64),
                drift=None if drift is None else np.ascontiguousarray(drift, dtype=np.float64),
                target_part=np.ascontiguousarray(target_part, dtype=np.int16),
                n_parts=int(n_parts), name=name, meta=dict(meta or {}))
    p.validate()
    return p


def _ball_sectors_2d(X, Y, centre, r, R):
    dx, dy = X - centre[0], Y - centre[1]
    inside = dx * dx + dy * dy <= r * r
    th = np.arctan2(dy, dx)
    th = np.where(th < 0.0, th + 2.0 * math.pi, th)
    part = np.minimum(R - 1, np.floor(R * th / (2.0 * math.pi)).astype(np.int64))
    return np.where(inside, part, -1).astype(np.int16)


def eikonal_2d(n: int = 101, nc: int = 32, r: float = 0.1, R: int = 1,
               centre=(0.0, 0.0), fp32: bool = False, name: str = "eikonal2d",
               h: Optional[float] = None) -> Problem:
    """f = a, A = N_c unit directions, target = ball of radius r, [-1,1]^2,
    h = k unless given.  The target is split into R equal-angle sectors."""
    lo, hi = (-1.0, -1.0), (1.0, 1.0)
    k = 2.0 / (n - 1)
    X, Y = grid_coords(2, (n, n), lo, hi)
    tp = _ball_sectors_2d(X, Y, centre, r, R)
    return _make(2, (n, n), k if h is None else h, unit_controls_2d(nc), np.ones(n * n), None, tp,
                 R, fp32, name, meta=dict(r=r, centre=tuple(centre), c=1.0))


def config1() -> Problem:
    """2D eikonal, 101^2 on [-1,1]^2, 32 controls, target ball r = 0.1 at the
    origin, h = k = 0.02, FP64; closed form T = |x| - 0.1."""
    return eikonal_2d(101, 32, 0.1, 1, (0.0, 0.0), fp32=False, name="config1-eikonal-101")


def coarse_size_2d(n: int, ratio: int = 16, lo: int = 17, hi: int = 65) -> int:
    return int(min(hi, max(lo, round((n - 1) / ratio) + 1)))


def variable_speed_2d(seed: int, n: int = 1025, nc_coarse: int = 65, nc: int = 32, R: int = 16,
                      r: float = 0.1, fp32: bool = True, drift_sign: Optional[int] = None,
                      name: str = "varspeed2d"):
    """Speed c = 1 + 0.5 sin(2 pi k1 x) sin(2 pi k2 y), (k1,k2) in {1,2,3}
    from the seed; target ball r centred at a seeded point in [-0.5,0.5]^2,
    split into R equal-angle parts.  Returns (fine, coarse).  With
    ``drift_sign`` set, adds the Zermelo-type drift
    w = 0.3 s (-sin(pi y), sin(pi x))."""
    rng = np.random.default_rng(seed)
    k1, k2 = (int(v) for v in rng.integers(1, 4, 2))
    centre = tuple(float(v) for v in rng.uniform(-0.5, 0.5, 2))
    out = []
    for nn, is_fp32 in ((n, fp32), (nc_coarse, False)):
        lo, hi = (-1.0, -1.0), (1.0, 1.0)
        kk = 2.0 / (nn - 1)
        X, Y = grid_coords(2, (nn, nn), lo, hi)
        # sines of each axis once, broadcast over the grid (the same values
        # and products as evaluating them node by node)
        ax = lo[0] + kk * np.arange(nn, dtype=np.float64)
        sx, sy = np.sin(2.0 * math.pi * k1 * ax), np.sin(2.0 * math.pi * k2 * ax)
        c = (1.0 + 0.5 * sx[None, :] * sy[:, None]).ravel()
        w = None
        if drift_sign is not None:
            wy = np.broadcast_to(-np.sin(math.pi * ax)[:, None], (nn, nn)).ravel()
            wx = np.broadcast_to(np.sin(math.pi * ax)[None, :], (nn, nn)).ravel()
            w = 0.3 * drift_sign * np.stack([wy, wx], axis=1)
        tp = _ball_sectors_2d(X, Y, centre, r, R)
        out.append(_make(2, (nn, nn), kk, unit_controls_2d(nc), c, w, tp, R, is_fp32,
                         f"{name}-s{seed}-n{nn}",
                         meta=dict(seed=seed, k1=k1, k2=k2, centre=centre, r=r)))
    return out[0], out[1]


def config2(seed: int = 0, n: int = 1025, nc_coarse: int = 65):
    """2D variable-speed patchy problem, 1025^2 fine / 65^2 coarse, 32
    controls, 16 equal-angle target parts (fine instance FP32-ready)."""
    return variable_speed_2d(seed, n, nc_coarse, 32, 16, 0.1, True, None, "config2")


def _sphere_parts(X, Y, Z, centre, r, bands, sectors):
    dx, dy, dz = X - centre[0], Y - centre[1], Z - centre[2]
    rr = dx * dx + dy * dy + dz * dz
    inside = rr <= r * r
    out = np.full(X.shape, -1, dtype=np.int16)
    # parts of the nodes inside the ball only (the rest stays -1)
    dx, dy, dz, rr = dx[inside], dy[inside], dz[inside], rr[inside]
    rad = np.sqrt(rr)
    uz = np.where(rad > 0.0, dz / np.where(rad > 0.0, rad, 1.0), 1.0)
    band = np.minimum(bands - 1, np.floor(bands * (1.0 - uz) / 2.0).astype(np.int64))
    th = np.arctan2(dy, dx)
    th = np.where(th < 0.0, th + 2.0 * math.pi, th)
    sec = np.minimum(sectors - 1, np.floor(sectors * th / (2.0 * math.pi)).astype(np.int64))
    part = band * sectors + sec
    out[inside] = np.where(rad > 0.0, part, 0).astype(np.int16)
    return out


def sphere_target_nodes(n: int, r: float = 0.15) -> int:
    """Number of nodes of the n^3 grid on [-1,1]^3 inside the ball of radius
    r at the origin (the target of the 3D variable-speed generator)."""
    X, Y, Z = grid_coords(3, (n, n, n), (-1.0,) * 3, (1.0,) * 3)
    return int((X * X + Y * Y + Z * Z <= r * r).sum())


def variable_speed_3d(seed: int, n: int = 257, nc_coarse: int = 33, nc: int = 98,
                      bands: int = 8, sectors: int = 8, r: float = 0.15, fp32: bool = True,
                      name: str = "varspeed3d"):
    """Speed c = 1 + 0.4 prod_i sin(2 pi k_i x_i), k_i in {1,2} from the
    seed; 98 Fibonacci directions; target ball r at the origin split into
    ``bands`` equal-area z-bands x ``sectors`` azimuth sectors."""
    rng = np.random.default_rng(seed)
    ks = [int(v) for v in rng.integers(1, 3, 3)]
    R = bands * sectors
    out = []
    for nn, is_fp32 in ((n, fp32), (nc_coarse, False)):
        lo, hi = (-1.0,) * 3, (1.0,) * 3
        kk = 2.0 / (nn - 1)
        X, Y, Z = grid_coords(3, (nn, nn, nn), lo, hi)
        # the sines of each axis once, broadcast over the grid (the same
        # values and products as evaluating them node by node)
        ax = lo[0] + kk * np.arange(nn, dtype=np.float64)
        sx, sy, sz = (np.sin(2.0 * math.pi * ks[d] * ax) for d in range(3))
        c = (1.0 + 0.4 * (sx[None, None, :] * sy[None, :, None] * sz[:, None, None])).ravel()
        tp = _sphere_parts(X, Y, Z, (0.0, 0.0, 0.0), r, bands, sectors)
        out.append(_make(3, (nn, nn, nn), kk, fibonacci_controls_3d(nc), c, None, tp, R, is_fp32,
                         f"{name}-s{seed}-n{nn}", meta=dict(seed=seed, ks=ks, r=r)))
    return out[0], out[1]


def config3(seed: int = 0, n: int = 257, nc_coarse: int = 33):
    """3D variable-speed patchy problem, 257^3 / 33^3, 98 controls, 64 parts."""
    return variable_speed_3d(seed, n, nc_coarse, 98, 8, 8, 0.15, True, "config3")


def eikonal_3d(n: int = 33, nc: int = 98, r: float = 0.3, bands: int = 1, sectors: int = 1,
               fp32: bool = False, name: str = "eikonal3d") -> Problem:
    lo, hi = (-1.0,) * 3, (1.0,) * 3
    kk = 2.0 / (n - 1)
    X, Y, Z = grid_coords(3, (n, n, n), lo, hi)
    tp = _sphere_parts(X, Y, Z, (0.0, 0.0, 0.0), r, bands, sectors)
    return _make(3, (n, n, n), kk, fibonacci_controls_3d(nc), np.ones(n ** 3), None, tp,
                 bands * sectors, fp32, name, meta=dict(r=r, c=1.0))


def line_target_2d(n: int = 41, nc: int = 32, col: Optional[int] = None, strips: int = 1,
                   fp32: bool = False, name: str = "line2d") -> Problem:
    """Target = one grid column {x = x_col}; with ``strips`` > 1 the column is
    split into that many horizontal strips (parts) of equal node count."""
    col = n // 2 if col is None else col
    lo, hi = (-1.0, -1.0), (1.0, 1.0)
    kk = 2.0 / (n - 1)
    tp = np.full((n, n), -1, dtype=np.int16)
    rows = np.arange(n)
    tp[:, col] = np.minimum(strips - 1, rows * strips // n).astype(np.int16)
    return _make(2, (n, n), kk, unit_controls_2d(nc), np.ones(n * n), None, tp.ravel(), strips,
                 fp32, name, meta=dict(col=col))


def with_obstacles(P: Problem, mask: np.ndarray, name: Optional[str] = None) -> Problem:
    """A copy of P whose nodes in `mask` (off the target) are obstacle nodes
    (target_part -2): a state constraint inside the box."""
    tp = P.target_part.copy()
    tp[np.asarray(mask).ravel() & (tp < 0)] = -2
    return dataclasses.replace(P, target_part=tp, name=name or P.name + "-obst")


def obstacle_mask_2d(X, Y, disc=(0.45, 0.3, 0.2), rect=(-0.75, -0.45, -0.6, 0.5)):
    """One disc (cx, cy, r) and one rectangle (x0, x1, y0, y1), the shapes of
    the paper's obstacle example."""
    cx, cy, r = disc
    x0, x1, y0, y1 = rect
    return ((X - cx) ** 2 + (Y - cy) ** 2 <= r * r) | ((X >= x0) & (X <= x1) & (Y >= y0) & (Y <= y1))


def eikonal_obstacles_2d(n: int = 129, nc: int = 32, R: int = 8, fp32: bool = False,
                         nc_coarse: int = 33):
    """Eikonal dynamics around a disc and a rectangle (Section 4.5), target
    ball r = 0.1 at the origin split into R sectors.  Returns (fine, coarse)
    with the obstacles on both grids."""
    out = []
    for nn, is32 in ((n, fp32), (nc_coarse, False)):
        P = eikonal_2d(nn, nc, 0.1, R, fp32=is32, name=f"obst2d-{nn}")
        X, Y = P.coords()
        out.append(with_obstacles(P, obstacle_mask_2d(X, Y).ravel()))
    return out[0], out[1]


def unit_reach(P: Problem, fp32: Optional[bool] = None) -> Problem:
    """The paper's variable step (Section 2.1): h_i = k / |f(x_i, a)| so that
    every foot point lies one cell away.  For drift-free dynamics
    f = c(x) a with unit controls on a grid of equal spacing k, the foot
    point is p + a_k (in cells) and beta_i = exp(-k / c_i) (0 where c_i = 0:
    the node cannot move).  Returns the problem with speed 1, step 1 and the
    per-node beta; the scalar beta becomes exp(-k)."""
    assert P.drift is None, "the variable step is built for drift-free dynamics"
    k = P.k[:P.dim]
    assert max(k) - min(k) <= 1e-12 * max(k), "equal grid spacing required"
    assert np.allclose(np.linalg.norm(P.controls, axis=1), 1.0, rtol=0, atol=1e-12)
    kk = float(k[0])
    fp32 = (P.meta.get("fp32", False) if fp32 is None else fp32)
    c = P.speed
    with np.errstate(divide="ignore"):
        bn = np.where(c > 0.0, np.exp(-kk / np.where(c > 0.0, c, 1.0)), 0.0)
    if fp32:
        bn = bn.astype(np.float32).astype(np.float64)
    b = _beta(kk, fp32)
    return dataclasses.replace(
        P, h=kk, step=(1.0, 1.0, 1.0 if P.dim == 3 else 0.0), beta=b, omb=1.0 - b,
        speed=np.ones(P.N), beta_node=np.ascontiguousarray(bn),
        name=P.name + "-unit", meta={**P.meta, "unit_reach": True, "c": c})


def _line_parts(n_other, R):
    """R strips of equal node count along the other axis (line targets)."""
    return np.minimum(R - 1, np.arange(n_other) * R // n_other).astype(np.int16)


def fan_2d(n: int = 101, nc: int = 32, R: int = 16, fp32: bool = False) -> Problem:
    """Fan dynamics of Table test2d: f = |x1 + x2 + 0.1| a on [-2,2]^2, unit
    controls, target the line {x1 = 0} split into R strips; with the paper's
    variable step (unit_reach).  n must be odd (a node column at x1 = 0)."""
    assert n % 2 == 1
    lo, hi = (-2.0, -2.0), (2.0, 2.0)
    k = 4.0 / (n - 1)
    X, Y = grid_coords(2, (n, n), lo, hi)
    tp = np.full((n, n), -1, dtype=np.int16)
    tp[:, (n - 1) // 2] = _line_parts(n, R)
    c = np.abs(X + Y + 0.1)
    P = _make(2, (n, n), k, unit_controls_2d(nc), c.ravel(), None, tp.ravel(), R, fp32,
              f"fan2d-{n}", lo=lo, hi=hi, meta=dict(fp32=fp32))
    return unit_reach(P, fp32)


def fan_3d(n: int = 33, nc: int = 189, R: int = 8, fp32: bool = False) -> Problem:
    """Fan 3D of Table test3d: f = |x1 + x2 + x3 + 0.1| a on [-2,2]^3,
    quasi-uniform unit controls, target the plane {x1 = 0} split into R
    blocks; with the paper's variable step.  n must be odd."""
    assert n % 2 == 1
    lo, hi = (-2.0, -2.0, -2.0), (2.0, 2.0, 2.0)
    k = 4.0 / (n - 1)
    X, Y, Z = grid_coords(3, (n, n, n), lo, hi)
    tp = np.full((n, n, n), -1, dtype=np.int16)
    ry = max(1, int(round(math.sqrt(R))))
    while R % ry:
        ry -= 1
    rz = R // ry
    py = _line_parts(n, ry).astype(np.int32)
    pz = _line_parts(n, rz).astype(np.int32)
    tp[:, :, (n - 1) // 2] = (pz[:, None] * ry + py[None, :]).astype(np.int16)
    c = np.abs(X + Y + Z + 0.1)
    P = _make(3, (n, n, n), k, fibonacci_controls_3d(nc), c.ravel(), None, tp.ravel(), R, fp32,
              f"fan3d-{n}", lo=lo, hi=hi, meta=dict(fp32=fp32))
    return unit_reach(P, fp32)


def eikonal_paper_2d(n: int = 101, nc: int = 32, R: int = 16, fp32: bool = False) -> Problem:
    """Eikonal of Table test2d: f = a on [-2,2]^2, target B(0, 0.5) split
    into R equal-angle sectors (the variable step is the constant h = k)."""
    lo, hi = (-2.0, -2.0), (2.0, 2.0)
    k = 4.0 / (n - 1)
    X, Y = grid_coords(2, (n, n), lo, hi)
    tp = _ball_sectors_2d(X, Y, (0.0, 0.0), 0.5, R)
    return _make(2, (n, n), k, unit_controls_2d(nc), np.ones(n * n), None, tp, R, fp32,
                 f"eikonal-paper-{n}", lo=lo, hi=hi, meta=dict(r=0.5, c=1.0))


def tabulate(P: Problem, f, fp32: bool = False) -> Problem:
    """Tabulated dynamics with the step rule of Section 2.1: for every node p
    and control k, h = k / |f(x_p, a_k)| puts the foot point one cell away,
    so the table holds the displacement f / |f| (in cells; equal grid
    spacing k) and beta = exp(-k / |f|); where f vanishes, displacement 0 and
    beta 0 (no move).  f(X, a) takes the node coordinates [N, dim] and one
    control [dim] and returns [N, dim]."""
    k = P.k[:P.dim]
    assert max(k) - min(k) <= 1e-12 * max(k), "equal grid spacing required"
    kk = float(k[0])
    X = np.stack(P.coords(), axis=1)
    foot = np.zeros((P.n_controls, P.N, P.dim))
    bpk = np.zeros((P.n_controls, P.N))
    for i, a in enumerate(P.controls):
        F = np.broadcast_to(np.asarray(f(X, a), dtype=np.float64), (P.N, P.dim))
        nf = np.linalg.norm(F, axis=1)
        ok = nf > 0.0
        foot[i, ok, :] = F[ok] / nf[ok, None]
        bpk[i, ok] = np.exp(-kk / nf[ok])
    if fp32:
        bpk = bpk.astype(np.float32).astype(np.float64)
    b = _beta(kk, fp32)
    return dataclasses.replace(
        P, h=kk, step=(1.0, 1.0, 1.0 if P.dim == 3 else 0.0), beta=b, omb=1.0 - b,
        speed=np.ones(P.N), drift=None, beta_node=None, foot=np.ascontiguousarray(foot),
        beta_pk=np.ascontiguousarray(bpk), name=P.name + "-tab", meta={**P.meta, "tabulated": True})


def eikonal_paper_3d(n: int = 51, nc: int = 189, R: int = 8, fp32: bool = False) -> Problem:
    """Eikonal 3D of Table test3d: f = a on [-2,2]^3, nc quasi-uniform unit
    controls, target B(0, 0.5) in R parts (2 bands x R/2 sectors)."""
    lo, hi = (-2.0,) * 3, (2.0,) * 3
    k = 4.0 / (n - 1)
    X, Y, Z = grid_coords(3, (n, n, n), lo, hi)
    tp = _sphere_parts(X, Y, Z, (0.0, 0.0, 0.0), 0.5, 2, max(1, R // 2))
    return _make(3, (n, n, n), k, fibonacci_controls_3d(nc), np.ones(n ** 3), None, tp,
                 2 * max(1, R // 2), fp32, f"eikonal-paper-3d-{n}", lo=lo, hi=hi,
                 meta=dict(r=0.5, c=1.0))


def zermelo_paper_2d(n: int = 101, nc: int = 32, R: int = 16, fp32: bool = False) -> Problem:
    """Zermelo of Table test2d: f = 2.1 a + (2, 0) on [-2,2]^2, unit
    controls, target B(0, 0.5) in R sectors, with the paper's step rule
    (per node and control, tabulated)."""
    P = eikonal_paper_2d(n, nc, R, fp32)
    P = dataclasses.replace(P, name=f"zermelo-paper-{n}", meta={**P.meta, "c": 2.1, "w": (2.0, 0.0)})
    return tabulate(P, lambda X, a: 2.1 * a[None, :] + np.array([2.0, 0.0])[None, :], fp32)


def brockett_3d(n: int = 33, R: int = 8, fp32: bool = False) -> Problem:
    """Brockett's integrator of Table test3d: f = (a1, a2, x1 a2 - x2 a1) on
    [-2,2]^3, A = {-5, 0, 5}^2 (9 controls, stored as (a1, a2, 0)), target
    B(0, 0.25) in R parts (2 bands x R/2 sectors), with the paper's step rule
    (tabulated)."""
    lo, hi = (-2.0, -2.0, -2.0), (2.0, 2.0, 2.0)
    k = 4.0 / (n - 1)
    assert k <= 0.25, "the target ball must hold nodes"
    X, Y, Z = grid_coords(3, (n, n, n), lo, hi)
    tp = _sphere_parts(X, Y, Z, (0.0, 0.0, 0.0), 0.25, 2, max(1, R // 2))
    ctrl = np.array([[a1, a2, 0.0] for a2 in (-5.0, 0.0, 5.0) for a1 in (-5.0, 0.0, 5.0)])
    P = _make(3, (n, n, n), k, ctrl, np.ones(n ** 3), None, tp, 2 * max(1, R // 2), fp32,
              f"brockett3d-{n}", lo=lo, hi=hi, meta=dict(r=0.25))

    def f(Xn, a):
        return np.stack([np.full(len(Xn), a[0]), np.full(len(Xn), a[1]),
                         Xn[:, 0] * a[1] - Xn[:, 1] * a[0]], axis=1)
    return tabulate(P, f, fp32)


def lunar_landing_2d(n: int = 101, eps: float = 0.12, R: int = 4, fp32: bool = False) -> Problem:
    """Lunar landing (Section 4.6): f = (x2, a), A = {-1, 1} (stored as
    (0, -1), (0, 1)), target B(0, eps) in R sectors, on [-1,1]^2, with the
    paper's step rule (tabulated)."""
    lo, hi = (-1.0, -1.0), (1.0, 1.0)
    k = 2.0 / (n - 1)
    X, Y = grid_coords(2, (n, n), lo, hi)
    tp = _ball_sectors_2d(X, Y, (0.0, 0.0), eps, R)
    ctrl = np.array([[0.0, -1.0], [0.0, 1.0]])
    P = _make(2, (n, n), k, ctrl, np.ones(n * n), None, tp, R, fp32, f"lunar-{n}",
              lo=lo, hi=hi, meta=dict(eps=eps))
    return tabulate(P, lambda Xn, a: np.stack([Xn[:, 1], np.full(len(Xn), a[1])], axis=1), fp32)


def zermelo_2d(n: int = 101, nc: int = 64, c: float = 1.0, w=(0.4, 0.0), r: float = 0.2,
               fp32: bool = False, name: str = "zermelo2d") -> Problem:
    """Constant-drift Zermelo problem f = c a + w (|w| < c), target ball r at
    the origin (cf. Table test2d, Zermelo)."""
    lo, hi = (-1.0, -1.0), (1.0, 1.0)
    kk = 2.0 / (n - 1)
    X, Y = grid_coords(2, (n, n), lo, hi)
    tp = _ball_sectors_2d(X, Y, (0.0, 0.0), r, 1)
    drift = np.tile(np.asarray(w, dtype=np.float64), (n * n, 1))
    return _make(2, (n, n), kk, unit_controls_2d(nc), np.full(n * n, float(c)), drift, tp, 1,
                 fp32, name, meta=dict(c=c, w=tuple(w), r=r))


def batched_problem(seed_seq: np.random.SeedSequence, index: int = 0,
                    n_range=(65, 769), nc_range=(16, 64), R_range=(4, 32)):
    """One problem of the batched workload: uneven grid side, control count
    and patch count; C2-type speed and target with a seeded-sign Zermelo
    drift.  Returns (fine, coarse)."""
    rng = np.random.default_rng(seed_seq)
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    nc = int(rng.integers(nc_range[0], nc_range[1] + 1))
    R = int(rng.integers(R_range[0], R_range[1] + 1))
    sign = int(rng.choice([-1, 1]))
    sub = int(rng.integers(0, 2 ** 31 - 1))
    ncoarse = coarse_size_2d(n)
    f, c = variable_speed_2d(sub, n, ncoarse, nc, R, 0.1, True, sign, f"batch{index}")
    f.meta.update(batch_index=index, drift_sign=sign)
    return f, c


def config4(count: int = 512, base_seed: int = 0, n_range=(65, 769)):
    """The batched workload: ``count`` independent 2D problems."""
    children = np.random.SeedSequence(base_seed).spawn(count)
    return [batched_problem(s, i, n_range) for i, s in enumerate(children)]


@dataclasses.dataclass
class ServingRequest:
    rid: int
    arrival_s: float
    fine: Problem
    coarse: Problem


def serving_specs(count: int, rate_per_s: float, seed: int = 0,
                  n2d=(129, 1025), n3d=(65, 193), frac3d: float = 0.2):
    """The random draws of the serving stream, request by request:
    (rid, arrival time, kind, sub-seed, grid side), kind 3 for the 3D
    variable-speed generator, 1 for the 2D eikonal, 4 for the batched 2D
    generator.  Cheap; serving_request builds the arrays of one spec."""
    rng = np.random.default_rng(seed)
    t = 0.0
    for i in range(count):
        t += float(rng.exponential(1.0 / rate_per_s))
        u = float(rng.uniform())
        sub = int(rng.integers(0, 2 ** 31 - 1))
        if u < frac3d:
            kind, n = 3, int(rng.integers(n3d[0], n3d[1] + 1))
        elif u < frac3d + (1.0 - frac3d) / 2.0:
            kind, n = 1, int(rng.integers(n2d[0], n2d[1] + 1))
        else:
            kind, n = 4, int(rng.integers(n2d[0], n2d[1] + 1))
        yield (i, t, kind, sub, n)


def serving_request(spec) -> "ServingRequest":
    """The request of one serving spec: 80% 2D (half eikonal with 16 sector
    parts, half the batched generator), 20% 3D (the 3D variable-speed
    generator with R = min(64, max(8, target nodes / 16)))."""
    i, t, kind, sub, n = spec
    if kind == 3:
        ncoarse = int(min(33, max(9, round((n - 1) / 8) + 1)))
        srng = np.random.default_rng(sub)
        ks_seed = int(srng.integers(0, 2 ** 31 - 1))
        R = int(min(64, max(8, sphere_target_nodes(n, 0.15) // 16)))
        bands, sectors = 8, 8
        if R != 64:
            bands = max(1, int(round(math.sqrt(R))))
            sectors = max(1, R // bands)
        f, c = variable_speed_3d(ks_seed, n, ncoarse, 98, bands, sectors, 0.15, True, f"req{i}")
    elif kind == 1:
        f = eikonal_2d(n, 32, 0.1, 16, (0.0, 0.0), True, f"req{i}")
        c = eikonal_2d(coarse_size_2d(n), 32, 0.1, 16, (0.0, 0.0), False, f"req{i}-c")
    else:
        f, c = batched_problem(np.random.SeedSequence(sub), i, (n, n))
    return ServingRequest(i, t, f, c)


def serving_stream(count: int, rate_per_s: float, seed: int = 0,
                   n2d=(129, 1025), n3d=(65, 193), frac3d: float = 0.2):
    """Poisson arrivals of solve requests: ``1 - frac3d`` 2D (half eikonal
    with 16 sector parts, half the batched generator), ``frac3d`` 3D (the 3D
    variable-speed generator).  Returns a generator of ServingRequest."""
    for spec in serving_specs(count, rate_per_s, seed, n2d, n3d, frac3d):
        yield serving_request(spec)
