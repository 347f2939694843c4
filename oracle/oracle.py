"""ctypes wrapper of the CPU FP64 oracle (hjb_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It shares
no code with the GPU path; the only common module is the seeded input
generator ``paper_1109_3577_amd.problems``, which carries no arithmetic of
the scheme.

Each function follows one step of the Patchy Algorithm (Section 3 of the
paper) or the SL value iteration of Section 2.1; the arithmetic lives in C.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hjb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMEM, ENOCONV = 0, 1, 3, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: FP64, no contraction, no fast-math."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wno-unknown-pragmas",
               _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Prob(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("step", C.c_double * 3),
                ("beta", C.c_double), ("omb", C.c_double), ("n_controls", C.c_int32),
                ("controls", C.c_void_p), ("speed", C.c_void_p), ("drift", C.c_void_p),
                ("target_part", C.c_void_p), ("n_parts", C.c_int32),
                ("beta_node", C.c_void_p), ("foot", C.c_void_p), ("beta_pk", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        vp, i32, d = C.c_void_p, C.c_int32, C.c_double
        L.orc_apply_F.argtypes = [vp, vp, i32, vp, vp]
        L.orc_F_at.argtypes = [vp, vp, i32, vp, vp, C.c_longlong, vp]
        L.orc_solve_global.argtypes = [vp, d, i32, vp, vp, vp, vp]
        L.orc_prolong.argtypes = [vp, vp, vp, vp]
        L.orc_feedback.argtypes = [vp, vp, vp]
        L.orc_feedback_at.argtypes = [vp, vp, vp, C.c_longlong, vp]
        L.orc_trace_part.argtypes = [vp, vp, i32, i32, vp, vp]
        L.orc_trace_part_mode.argtypes = [vp, vp, i32, i32, i32, vp, vp]
        L.orc_labels.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
        L.orc_detach_fragments.argtypes = [vp, vp, vp]
        L.orc_fill_labels.argtypes = [vp, vp, vp]
        L.orc_solve_patches.argtypes = [vp, vp, d, i32, i32, vp, vp, vp]
        L.orc_solve_patches_ex.argtypes = [vp, vp, vp, d, vp, vp, d, i32, i32, vp, vp, vp]
        L.orc_cone_allowed.argtypes = [vp, d, vp]
        L.orc_exclude.argtypes = [vp, vp, d, vp]
        L.orc_F_at_ex.argtypes = [vp, vp, i32, vp, d, vp, vp, vp, C.c_longlong, vp]
        L.orc_exclude.restype = C.c_longlong
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


class _Held:
    """A ctypes problem struct plus the arrays it points into."""

    def __init__(self, P):
        self.arrays = []
        s = _Prob()
        s.dim = P.dim
        for d in range(3):
            s.n[d] = int(P.n[d])
            s.step[d] = float(P.step[d])
        s.beta = float(P.beta)
        s.omb = float(P.omb)
        s.n_controls = int(P.controls.shape[0])
        s.controls = self._ptr(P.controls, np.float64)
        s.speed = self._ptr(P.speed, np.float64)
        s.drift = None if P.drift is None else self._ptr(P.drift, np.float64)
        s.target_part = self._ptr(P.target_part, np.int16)
        s.n_parts = int(P.n_parts)
        bn = getattr(P, "beta_node", None)
        s.beta_node = None if bn is None else self._ptr(bn, np.float64)
        ft, bp = getattr(P, "foot", None), getattr(P, "beta_pk", None)
        s.foot = None if ft is None else self._ptr(ft, np.float64)
        s.beta_pk = None if bp is None else self._ptr(bp, np.float64)
        self.s = s

    def _ptr(self, a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        self.arrays.append(a)
        return a.ctypes.data

    @property
    def ref(self):
        return C.byref(self.s)


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _check(rc, what, allow_noconv=False):
    if rc == OK or (allow_noconv and rc == ENOCONV):
        return
    raise RuntimeError(f"oracle {what} failed with status {rc}")


def set_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def apply_F(P, v_in: np.ndarray, labels: Optional[np.ndarray] = None, patch: int = -1):
    """One raw application of F (Section 2.1), every node."""
    H = _Held(P)
    v_in = np.ascontiguousarray(v_in, dtype=np.float64).ravel()
    out = np.empty_like(v_in)
    lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.int16).ravel()
    _check(lib().orc_apply_F(H.ref, _p(lab), int(patch), _p(v_in), _p(out)), "apply_F")
    return out


def F_at(P, v: np.ndarray, idx: np.ndarray, labels: Optional[np.ndarray] = None, patch: int = -1):
    """F evaluated at the listed nodes only, for node-by-node checks."""
    H = _Held(P)
    v = np.ascontiguousarray(v, dtype=np.float64).ravel()
    idx = np.ascontiguousarray(idx, dtype=np.int64).ravel()
    out = np.empty(idx.shape[0], dtype=np.float64)
    lab = None if labels is None else np.ascontiguousarray(labels, dtype=np.int16).ravel()
    _check(lib().orc_F_at(H.ref, _p(lab), int(patch), _p(v), _p(idx), idx.shape[0], _p(out)),
           "F_at")
    return out


def F_at_ex(P, v: np.ndarray, idx: np.ndarray, labels: np.ndarray, patch: int,
            fb: Optional[np.ndarray] = None, r: float = 0.0, u0: Optional[np.ndarray] = None):
    """F of patch `patch` at the listed nodes with the add-on options (AO3
    cones around fb for r > 1, Dirichlet data u0)."""
    H = _Held(P)
    v = np.ascontiguousarray(v, dtype=np.float64).ravel()
    idx = np.ascontiguousarray(idx, dtype=np.int64).ravel()
    out = np.empty(idx.shape[0], dtype=np.float64)
    lab = np.ascontiguousarray(labels, dtype=np.int16).ravel()
    fbc = None if fb is None else np.ascontiguousarray(fb, dtype=np.uint8).ravel()
    u0c = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64).ravel()
    _check(lib().orc_F_at_ex(H.ref, _p(lab), int(patch), _p(fbc), float(r), _p(u0c), _p(v),
                             _p(idx), idx.shape[0], _p(out)), "F_at_ex")
    return out


def solve_global(P, tol: float = 0.0, max_sweeps: int = 1_000_000, allow_noconv=False):
    """Value iteration eq. iterativeSLscheme, every node active, Jacobi."""
    H = _Held(P)
    v = np.empty(P.N, dtype=np.float64)
    sw, res, upd = C.c_int(0), C.c_double(0.0), C.c_longlong(0)
    rc = lib().orc_solve_global(H.ref, float(tol), int(max_sweeps), _p(v), C.byref(sw),
                                C.byref(res), C.byref(upd))
    _check(rc, "solve_global", allow_noconv)
    return v, dict(sweeps=sw.value, residual=res.value, updates=upd.value, status=rc)


def prolong(coarse, v_coarse: np.ndarray, fine):
    """Step 2: U_P^(0) = interpolation of the coarse solution on G."""
    Hc, Hf = _Held(coarse), _Held(fine)
    vc = np.ascontiguousarray(v_coarse, dtype=np.float64).ravel()
    u0 = np.empty(fine.N, dtype=np.float64)
    _check(lib().orc_prolong(Hc.ref, _p(vc), Hf.ref, _p(u0)), "prolong")
    return u0


def feedback(fine, u0: np.ndarray):
    """Step 2: discrete feedback a*_k~ at every fine node (255 on target)."""
    H = _Held(fine)
    u0 = np.ascontiguousarray(u0, dtype=np.float64).ravel()
    fb = np.empty(fine.N, dtype=np.uint8)
    _check(lib().orc_feedback(H.ref, _p(u0), _p(fb)), "feedback")
    return fb


def feedback_at(fine, u0: np.ndarray, idx: np.ndarray):
    """Step 2 feedback at the listed nodes only."""
    H = _Held(fine)
    u0 = np.ascontiguousarray(u0, dtype=np.float64).ravel()
    idx = np.ascontiguousarray(idx, dtype=np.int64).ravel()
    fb = np.empty(idx.shape[0], dtype=np.uint8)
    _check(lib().orc_feedback_at(H.ref, _p(u0), _p(idx), idx.shape[0], _p(fb)), "feedback_at")
    return fb


def trace_part(fine, fb: np.ndarray, part: int, max_sweeps: int = 1_000_000):
    """Step 3.1 for one part in the labels' reading (the colour lattice):
    the colour field phi^j at its fixed point."""
    H = _Held(fine)
    fb = np.ascontiguousarray(fb, dtype=np.uint8).ravel()
    phi = np.empty(fine.N, dtype=np.float64)
    sw = C.c_int(0)
    _check(lib().orc_trace_part(H.ref, _p(fb), int(part), int(max_sweeps), _p(phi), C.byref(sw)),
           "trace_part")
    return phi, sw.value


TRACE_DISCOUNTED, TRACE_PLAIN, TRACE_PAPER, TRACE_LATTICE = 0, 1, 2, 3
# spacing of the colour lattice of the labels' transport
COLOUR_LATTICE = 2.0 ** -24


def trace_part_mode(fine, fb: np.ndarray, part: int, mode: int, max_sweeps: int = 1_000_000,
                    allow_noconv: bool = False):
    """Step 3.1 for one part in one reading of eq. HJBridotta_discreta:
    TRACE_LATTICE (the labels' reading: scheme step, factor beta, colours
    rounded down to multiples of 2^-24), TRACE_DISCOUNTED (scheme step,
    factor beta, floor 1e-9, unrounded), TRACE_PLAIN (scheme step, no
    factor, no floor) or TRACE_PAPER (no factor, no floor, foot point one
    cell away along f).  Returns (phi, sweeps, status)."""
    H = _Held(fine)
    fb = np.ascontiguousarray(fb, dtype=np.uint8).ravel()
    phi = np.empty(fine.N, dtype=np.float64)
    sw = C.c_int(0)
    rc = lib().orc_trace_part_mode(H.ref, _p(fb), int(part), int(mode), int(max_sweeps), _p(phi),
                                   C.byref(sw))
    _check(rc, "trace_part_mode", allow_noconv)
    return phi, sw.value, rc


def labels(fine, fb: np.ndarray, max_sweeps: int = 1_000_000, want_sum: bool = False,
           want_unreached: bool = False, want_detached: bool = False):
    """Step 3.1 for every part plus the projection/assembly into labels:
    pieces of a patch cut off from their own target part are uncoloured, and
    every uncoloured node takes its neighbours' colour (Remark 3.1).
    want_sum adds (sum of colours, max sweeps of a part); want_unreached adds
    the number of nodes no colour reached; want_detached the number of nodes
    in cut-off pieces."""
    H = _Held(fine)
    fb = np.ascontiguousarray(fb, dtype=np.uint8).ravel()
    lab = np.empty(fine.N, dtype=np.int16)
    s = np.empty(fine.N, dtype=np.float64) if want_sum else None
    mx = C.c_int(0)
    un = C.c_longlong(0)
    de = C.c_longlong(0)
    _check(lib().orc_labels(H.ref, _p(fb), int(max_sweeps), _p(lab), _p(s), C.byref(mx),
                            C.byref(un), C.byref(de)), "labels")
    out = (lab,)
    if want_sum:
        out = out + (s, mx.value)
    if want_unreached:
        out = out + (un.value,)
    if want_detached:
        out = out + (de.value,)
    return out if len(out) > 1 else lab


def detach_fragments(fine, labels_: np.ndarray):
    """Remark 3.1 applied to cut-off pieces: the labels of every connected
    piece of one label (8 / 26 neighbours) without a target node of that
    label become -1.  Returns (new labels, number of nodes relabelled)."""
    H = _Held(fine)
    lab = np.array(labels_, dtype=np.int16).ravel()
    de = C.c_longlong(0)
    _check(lib().orc_detach_fragments(H.ref, _p(lab), C.byref(de)), "detach_fragments")
    return lab, de.value


def fill_labels(fine, labels_: np.ndarray):
    """Remark 3.1: every -1 node takes the lowest label among its nearest
    labelled nodes (layer by layer)."""
    H = _Held(fine)
    lab = np.array(labels_, dtype=np.int16).ravel()
    _check(lib().orc_fill_labels(H.ref, _p(lab), None), "fill_labels")
    return lab


def solve_patches(fine, labels_: np.ndarray, tol: float = 0.0, max_sweeps: int = 1_000_000,
                  only_patch: int = -1):
    """Steps 3.2 and 4: independent per-patch iteration and merge."""
    H = _Held(fine)
    lab = np.ascontiguousarray(labels_, dtype=np.int16).ravel()
    v = np.empty(fine.N, dtype=np.float64)
    sw = np.zeros(max(1, fine.n_parts), dtype=np.int32)
    upd = C.c_longlong(0)
    _check(lib().orc_solve_patches(H.ref, _p(lab), float(tol), int(max_sweeps), int(only_patch),
                                   _p(v), _p(sw), C.byref(upd)), "solve_patches")
    return v, dict(sweeps=sw, updates=upd.value)


def cone_allowed(fine, r: float):
    """Add-on AO3: allowed[ks, k] = 1 iff control k lies in the cone of
    half-angle pi/r around the feedback control ks.  Returns (allowed,
    largest set size)."""
    H = _Held(fine)
    nc = int(fine.controls.shape[0])
    allow = np.empty((nc, nc), dtype=np.uint8)
    lmax = lib().orc_cone_allowed(H.ref, float(r), _p(allow))
    if lmax < 0:
        raise RuntimeError("oracle cone_allowed failed")
    return allow, int(lmax)


def solve_patches_ex(fine, labels_: np.ndarray, fb: Optional[np.ndarray] = None, r: float = 0.0,
                     u0: Optional[np.ndarray] = None, tol: float = 0.0,
                     max_sweeps: int = 1_000_000, only_patch: int = -1,
                     init: Optional[np.ndarray] = None):
    """Steps 3.2 and 4 with the options of the paper's add-ons section:
    add-on AO3 (fb, r > 1: each node minimises over the controls in the cone
    of half-angle pi/r around its Step 2 feedback control), the Dirichlet
    patch boundary data of eq. dbc (u0: other patches' nodes hold U^(0)
    instead of the ghost value 1) and add-on AO1 (init: start values of the
    patch nodes, iteration v <- F(v), tol > 0)."""
    H = _Held(fine)
    lab = np.ascontiguousarray(labels_, dtype=np.int16).ravel()
    fbc = None if fb is None else np.ascontiguousarray(fb, dtype=np.uint8).ravel()
    u0c = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64).ravel()
    inc = None if init is None else np.ascontiguousarray(init, dtype=np.float64).ravel()
    v = np.empty(fine.N, dtype=np.float64)
    sw = np.zeros(max(1, fine.n_parts), dtype=np.int32)
    upd = C.c_longlong(0)
    _check(lib().orc_solve_patches_ex(H.ref, _p(lab), _p(fbc), float(r), _p(u0c), _p(inc),
                                      float(tol), int(max_sweeps), int(only_patch), _p(v),
                                      _p(sw), C.byref(upd)), "solve_patches_ex")
    return v, dict(sweeps=sw, updates=upd.value)


def solve_patches_cone(fine, labels_: np.ndarray, fb: np.ndarray, r: float, tol: float = 0.0,
                       max_sweeps: int = 1_000_000, only_patch: int = -1):
    """Steps 3.2 and 4 with add-on AO3 only."""
    return solve_patches_ex(fine, labels_, fb, r, None, tol, max_sweeps, only_patch)


def exclude(fine, u0: np.ndarray, theta: float):
    """Section 4.6: fine nodes off the target with U^(0) >= theta become
    obstacle nodes (-2).  Returns (new target_part, number excluded)."""
    H = _Held(fine)
    u0 = np.ascontiguousarray(u0, dtype=np.float64).ravel()
    tp = np.empty(fine.N, dtype=np.int16)
    n = lib().orc_exclude(H.ref, _p(u0), float(theta), _p(tp))
    if n < 0:
        raise RuntimeError("oracle exclude failed")
    return tp, int(n)


def patchy(fine, coarse, tol: float = 0.0, max_sweeps: int = 1_000_000,
           exclude_at: Optional[float] = None):
    """The whole Patchy Algorithm of Section 3, Steps 1-4.  With exclude_at,
    the unreachable regions (U^(0) >= exclude_at) are dropped after Step 1
    (Section 4.6) and become obstacle nodes of the fine problem."""
    import dataclasses
    vc, cst = solve_global(coarse, 0.0, max_sweeps)
    u0 = prolong(coarse, vc, fine)
    excluded = 0
    if exclude_at is not None:
        tp, excluded = exclude(fine, u0, exclude_at)
        fine = dataclasses.replace(fine, target_part=tp)
        u0 = prolong(coarse, vc, fine)
    fb = feedback(fine, u0)
    lab = labels(fine, fb, max_sweeps)
    v, st = solve_patches(fine, lab, tol, max_sweeps)
    return dict(v=v, labels=lab, feedback=fb, u0=u0, v_coarse=vc, coarse_stats=cst, stats=st,
                excluded=excluded, target_part=fine.target_part)
