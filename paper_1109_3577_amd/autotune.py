"""Autotuner for the tiled sweep: tile shape, workgroup size and in-tile
sweeps per activation.

Every candidate runs the real solve through the C ABI (hjb_solve_patches on
a prepared patches handle, or a batch); since every schedule reaches the
same fixed point, the choice only moves time, never results.  Choices are
cached per (dimension, precision, size bucket, control bucket) in memory and
optionally in a JSON file.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional, Sequence, Tuple

from . import hjb

CANDIDATES = {
    2: [((32, 8, 1), 256), ((16, 16, 1), 256), ((64, 8, 1), 512), ((32, 16, 1), 512),
        ((32, 16, 1), 256), ((32, 32, 1), 512)],
    3: [((8, 8, 8), 256), ((8, 8, 8), 512), ((16, 8, 8), 512)],
}
SWEEPS = {2: (8, 12, 16, 24), 3: (2, 4, 8)}

_cache: Dict[str, dict] = {}


def _key(dim: int, precision: int, N: int, nc: int) -> str:
    nb = 1
    while nb < N:
        nb *= 4
    cb = 16 if nc <= 16 else (32 if nc <= 32 else (64 if nc <= 64 else 128))
    return f"d{dim}-p{precision}-N{nb}-c{cb}"


def load(path: str) -> None:
    if os.path.exists(path):
        with open(path) as fh:
            _cache.update(json.load(fh))


def save(path: str) -> None:
    with open(path, "w") as fh:
        json.dump(_cache, fh, indent=1, sort_keys=True)


def opts_from(choice: dict, **extra) -> hjb.hjb_solve_opts:
    return hjb.make_opts(tile=choice["tile"], threads=choice["threads"],
                         inner_sweeps=choice["inner_sweeps"], **extra)


def tune_patches(fine, patches: "hjb.Patches", precision: int = hjb.HJB_F32, tol: float = 1e-5,
                 stream=None, repeats: int = 2, candidates: Optional[Sequence] = None,
                 sweeps: Optional[Sequence[int]] = None, verbose: bool = False) -> dict:
    """Times every candidate on one prepared problem; returns the fastest
    {"tile", "threads", "inner_sweeps", "ms"} and caches it."""
    import torch
    P = hjb._as_problem(fine)
    dim = P.s.dim
    v = torch.empty(P.N, dtype=torch.float32 if precision == hjb.HJB_F32 else torch.float64,
                    device="cuda")
    best = None
    for tile, nt in (candidates or CANDIDATES[dim]):
        for K in (sweeps or SWEEPS[dim]):
            o = hjb.make_opts(tile=tile, threads=nt, inner_sweeps=K)
            ts = []
            for _ in range(repeats):
                torch.cuda.synchronize()
                t = time.perf_counter()
                hjb.hjb_solve_patches(P, patches, precision, v, tol, 0, o, stream)
                ts.append((time.perf_counter() - t) * 1e3)
            ms = min(ts)
            if verbose:
                print(f"[autotune] tile {tile} threads {nt} K {K}: {ms:.2f} ms", flush=True)
            if best is None or ms < best["ms"]:
                best = {"tile": list(tile), "threads": nt, "inner_sweeps": K, "ms": ms}
    _cache[_key(dim, precision, P.N, P.s.n_controls)] = best
    return best


def lookup(dim: int, precision: int, N: int, nc: int) -> Optional[dict]:
    return _cache.get(_key(dim, precision, N, nc))


def tune_batch(fines: Sequence, coarses: Sequence, precision: int = hjb.HJB_F32,
               tol: float = 1e-5, sample: int = 8, verbose: bool = False,
               repeats: int = 2) -> Tuple[dict, float]:
    """Picks tile / threads / sweeps for a batch by timing hjb_batch_run on a
    sample of its problems (best of `repeats` runs, a fresh batch each);
    returns (choice, ms of the best sample run)."""
    step = max(1, len(fines) // sample)
    fs, cs = list(fines)[::step][:sample], list(coarses)[::step][:sample]
    dims = {hjb._as_problem(f).s.dim for f in fs}
    dim = 2 if dims == {2} else 3
    best = None
    for tile, nt in CANDIDATES[dim]:
        for K in SWEEPS[dim]:
            o = hjb.make_opts(tile=tile, threads=nt, inner_sweeps=K)
            ms = float("inf")
            for _ in range(max(1, repeats)):
                b = hjb.hjb_batch_create(fs, cs, precision, tol, 0, o)
                t = time.perf_counter()
                b.run()
                ms = min(ms, (time.perf_counter() - t) * 1e3)
                b.free()
            if verbose:
                print(f"[autotune] batch tile {tile} threads {nt} K {K}: {ms:.2f} ms", flush=True)
            if best is None or ms < best["ms"]:
                best = {"tile": list(tile), "threads": nt, "inner_sweeps": K, "ms": ms}
    return best, best["ms"]
