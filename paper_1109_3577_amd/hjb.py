"""Python binding of libhjb (include/hjb.h): argument marshalling only.

Every function here forwards to the C ABI function of the same name; all
computation runs in the library's HIP kernels.  PyTorch supplies device
memory (tensors) and the stream.  If the library is missing, importing this
module raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhjb.so")

HJB_OK, HJB_EINVAL, HJB_EDEVICE, HJB_ENOMEM, HJB_ENOCONV, HJB_EAGAIN = 0, 1, 2, 3, 4, 5
HJB_MEM_HOST, HJB_MEM_DEVICE = 0, 1
HJB_F32, HJB_F64 = 0, 1
HJB_SCHED_TILED, HJB_SCHED_JACOBI, HJB_SCHED_ASYNC = 0, 1, 2
HJB_BC_STATE, HJB_BC_DIRICHLET = 0, 1
HJB_OBSTACLE = -2
HJB_NOALLOC_MAX_NODES = 1 << 21

# Every symbol include/hjb.h declares.
EXPORTS = (
    "hjb_coarse_solve", "hjb_coarse_values", "hjb_coarse_free", "hjb_build_patches",
    "hjb_build_patches_ex",
    "hjb_patches_labels", "hjb_patches_feedback", "hjb_patches_u0", "hjb_patches_free",
    "hjb_solve_patches", "hjb_solve_global", "hjb_solve_global_noalloc", "hjb_batch_create",
    "hjb_batch_run",
    "hjb_batch_result", "hjb_batch_free", "hjb_server_create", "hjb_server_submit",
    "hjb_server_step", "hjb_server_poll", "hjb_server_free", "hjb_last_error", "hjb_version",
)


class hjb_problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("step", C.c_double * 3),
                ("beta", C.c_double), ("one_minus_beta", C.c_double),
                ("n_controls", C.c_int32), ("controls", C.c_void_p), ("speed", C.c_void_p),
                ("drift", C.c_void_p), ("target_part", C.c_void_p), ("n_parts", C.c_int32),
                ("mem", C.c_int32), ("beta_node", C.c_void_p), ("foot", C.c_void_p),
                ("beta_pk", C.c_void_p)]


class hjb_stats(C.Structure):
    _fields_ = [("updates", C.c_int64), ("node_updates", C.c_int64), ("item_runs", C.c_int64),
                ("items", C.c_int32), ("rounds", C.c_int32), ("residual", C.c_double),
                ("ms_wall", C.c_double), ("ms_kernel", C.c_double),
                ("kernel_launches", C.c_int32), ("status", C.c_int32),
                ("ms_prolong_feedback", C.c_double), ("ms_trace", C.c_double),
                ("trace_node_updates", C.c_int64), ("unreached", C.c_int32),
                ("sweeps", C.c_int32), ("tile", C.c_int32 * 3), ("threads", C.c_int32),
                ("inner_sweeps", C.c_int32), ("excluded", C.c_int32),
                ("detached", C.c_int32)]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            x = getattr(self, name)
            out[name] = list(x) if name == "tile" else x
        return out


class hjb_solve_opts(C.Structure):
    _fields_ = [("tile", C.c_int32 * 3), ("inner_sweeps", C.c_int32),
                ("rounds_per_poll", C.c_int32), ("schedule", C.c_int32),
                ("time_kernels", C.c_int32), ("use_graph", C.c_int32), ("threads", C.c_int32),
                ("patch_select", C.c_void_p), ("control_cone", C.c_double),
                ("patch_bc", C.c_int32), ("order_window", C.c_double),
                ("start_u0", C.c_int32)]


class hjb_build_opts(C.Structure):
    _fields_ = [("exclude_at", C.c_double)]


class hjb_batch_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("tol", C.c_double), ("max_sweeps", C.c_int32),
                ("solve", hjb_solve_opts), ("prepare_bytes", C.c_uint64)]


class hjb_server_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("tol", C.c_double), ("max_sweeps", C.c_int32),
                ("solve", hjb_solve_opts)]


class HjbError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: status {status}: {last_error()}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = C.CDLL(LIB_PATH)
    vp, i32, d, P = C.c_void_p, C.c_int32, C.c_double, C.POINTER
    L.hjb_last_error.restype = C.c_char_p
    L.hjb_version.restype = C.c_char_p
    L.hjb_coarse_solve.argtypes = [P(hjb_problem), d, i32, vp, P(vp)]
    L.hjb_coarse_values.argtypes = [vp, vp, i32]
    L.hjb_coarse_free.argtypes = [vp]
    L.hjb_coarse_free.restype = None
    L.hjb_build_patches.argtypes = [P(hjb_problem), vp, vp, P(vp), P(hjb_stats)]
    L.hjb_build_patches_ex.argtypes = [P(hjb_problem), vp, P(hjb_build_opts), vp, P(vp),
                                       P(hjb_stats)]
    for f in ("hjb_patches_labels", "hjb_patches_feedback", "hjb_patches_u0"):
        getattr(L, f).argtypes = [vp, vp, i32]
    L.hjb_patches_free.argtypes = [vp]
    L.hjb_patches_free.restype = None
    L.hjb_solve_patches.argtypes = [P(hjb_problem), vp, i32, d, i32, vp, P(hjb_solve_opts),
                                    P(hjb_stats), vp]
    L.hjb_solve_global.argtypes = [P(hjb_problem), i32, d, i32, vp, P(hjb_solve_opts),
                                   P(hjb_stats), vp]
    L.hjb_solve_global_noalloc.argtypes = [P(hjb_problem), i32, d, i32, vp, P(hjb_stats), vp]
    L.hjb_batch_create.argtypes = [P(P(hjb_problem)), P(P(hjb_problem)), i32, P(hjb_batch_opts),
                                   vp, P(vp)]
    L.hjb_batch_run.argtypes = [vp, vp, P(hjb_stats)]
    L.hjb_batch_result.argtypes = [vp, i32, vp, i32, P(hjb_stats)]
    L.hjb_batch_free.argtypes = [vp]
    L.hjb_batch_free.restype = None
    L.hjb_server_create.argtypes = [C.c_size_t, P(hjb_server_opts), vp, P(vp)]
    L.hjb_server_submit.argtypes = [vp, P(hjb_problem), P(hjb_problem), P(C.c_uint64)]
    L.hjb_server_step.argtypes = [vp, i32, P(i32), P(i32)]
    L.hjb_server_poll.argtypes = [vp, C.c_uint64, vp, i32, P(hjb_stats)]
    L.hjb_server_free.argtypes = [vp]
    L.hjb_server_free.restype = None
    return L


lib = _load()


def last_error() -> str:
    return lib.hjb_last_error().decode()


def hjb_version() -> str:
    return lib.hjb_version().decode()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(rc: int, what: str, ok=(HJB_OK,)) -> int:
    if rc not in ok:
        raise HjbError(rc, what)
    return rc


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


class Problem:
    """An hjb_problem plus the arrays it points to (kept alive here).

    ``source`` is a :class:`paper_1109_3577_amd.problems.Problem`;
    ``device=True`` copies its arrays to torch CUDA tensors (mem =
    HJB_MEM_DEVICE), otherwise host numpy arrays are passed (HJB_MEM_HOST)."""

    def __init__(self, source, device: bool = False):
        self.source = source
        self.keep = []
        s = hjb_problem()
        s.dim = source.dim
        for k in range(3):
            s.n[k] = int(source.n[k])
            s.step[k] = float(source.step[k])
        s.beta = float(source.beta)
        s.one_minus_beta = float(source.omb)
        s.n_controls = int(source.controls.shape[0])
        s.n_parts = int(source.n_parts)
        bn = getattr(source, "beta_node", None)
        ft, bp = getattr(source, "foot", None), getattr(source, "beta_pk", None)
        arrs = [np.ascontiguousarray(source.controls, dtype=np.float64),
                np.ascontiguousarray(source.speed, dtype=np.float64),
                None if source.drift is None else np.ascontiguousarray(source.drift, dtype=np.float64),
                np.ascontiguousarray(source.target_part, dtype=np.int16),
                None if bn is None else np.ascontiguousarray(bn, dtype=np.float64),
                None if ft is None else np.ascontiguousarray(ft, dtype=np.float64),
                None if bp is None else np.ascontiguousarray(bp, dtype=np.float64)]
        if device:
            import torch
            arrs = [None if a is None else torch.from_numpy(a).cuda() for a in arrs]
            s.mem = HJB_MEM_DEVICE
        else:
            s.mem = HJB_MEM_HOST
        self.keep = arrs
        (s.controls, s.speed, s.drift, s.target_part, s.beta_node, s.foot,
         s.beta_pk) = (_ptr(a) for a in arrs)
        self.s = s

    @property
    def ref(self):
        return C.byref(self.s)

    @property
    def N(self) -> int:
        return self.s.n[0] * self.s.n[1] * self.s.n[2]


def _as_problem(p, device=False) -> Problem:
    return p if isinstance(p, Problem) else Problem(p, device)


def make_opts(tile=None, inner_sweeps=0, rounds_per_poll=0, schedule=HJB_SCHED_TILED,
              time_kernels=False, use_graph=False, patch_select=None,
              threads=0, control_cone=0.0, patch_bc=0, order_window=0.0,
              start_u0=False) -> hjb_solve_opts:
    o = hjb_solve_opts()
    if tile is not None:
        for k, t in enumerate(tile):
            o.tile[k] = int(t)
    o.inner_sweeps = int(inner_sweeps)
    o.rounds_per_poll = int(rounds_per_poll)
    o.schedule = int(schedule)
    o.time_kernels = int(bool(time_kernels))
    o.use_graph = int(bool(use_graph))
    o.threads = int(threads)
    o.control_cone = float(control_cone)
    o.patch_bc = int(patch_bc)
    o.order_window = float(order_window)
    o.start_u0 = int(bool(start_u0))
    if patch_select is not None:
        sel = np.ascontiguousarray(patch_select, dtype=np.uint8)
        o._sel = sel
        o.patch_select = sel.ctypes.data
    return o


class Coarse:
    """Owning wrapper of an hjb_coarse_t handle."""

    def __init__(self, handle: int, n: int):
        self.h = handle
        self.N = n

    def values(self) -> np.ndarray:
        out = np.empty(self.N, dtype=np.float64)
        _check(lib.hjb_coarse_values(self.h, out.ctypes.data, HJB_MEM_HOST), "hjb_coarse_values")
        return out

    def free(self):
        if self.h and lib is not None:
            lib.hjb_coarse_free(self.h)
        self.h = None

    def __del__(self):
        self.free()


class Patches:
    """Owning wrapper of an hjb_patches_t handle."""

    def __init__(self, handle: int, n: int, stats: dict):
        self.h = handle
        self.N = n
        self.stats = stats

    def _get(self, fn, dtype):
        out = np.empty(self.N, dtype=dtype)
        _check(fn(self.h, out.ctypes.data, HJB_MEM_HOST), fn.__name__)
        return out

    def labels(self) -> np.ndarray:
        return self._get(lib.hjb_patches_labels, np.int16)

    def feedback(self) -> np.ndarray:
        return self._get(lib.hjb_patches_feedback, np.uint8)

    def u0(self) -> np.ndarray:
        return self._get(lib.hjb_patches_u0, np.float64)

    def free(self):
        if self.h and lib is not None:
            lib.hjb_patches_free(self.h)
        self.h = None

    def __del__(self):
        self.free()


def hjb_coarse_solve(coarse, tol: float = 0.0, max_sweeps: int = 0, stream=None,
                     device: bool = False, allow_noconv: bool = False) -> Coarse:
    P = _as_problem(coarse, device)
    h = C.c_void_p()
    rc = lib.hjb_coarse_solve(P.ref, float(tol), int(max_sweeps), _stream(stream), C.byref(h))
    _check(rc, "hjb_coarse_solve", (HJB_OK, HJB_ENOCONV) if allow_noconv else (HJB_OK,))
    return Coarse(h.value, P.N)


def hjb_build_patches(fine, coarse: Coarse, stream=None, device: bool = False,
                      exclude_at: Optional[float] = None) -> Patches:
    """Steps 2 and 3.1; with exclude_at, hjb_build_patches_ex (Section 4.6)."""
    P = _as_problem(fine, device)
    h = C.c_void_p()
    st = hjb_stats()
    if exclude_at is None:
        rc = lib.hjb_build_patches(P.ref, coarse.h, _stream(stream), C.byref(h), C.byref(st))
    else:
        o = hjb_build_opts()
        o.exclude_at = float(exclude_at)
        rc = lib.hjb_build_patches_ex(P.ref, coarse.h, C.byref(o), _stream(stream), C.byref(h),
                                      C.byref(st))
    _check(rc, "hjb_build_patches")
    return Patches(h.value, P.N, st.as_dict())


def hjb_solve_patches(fine, patches: Patches, precision: int, v_out, tol: float = 0.0,
                      max_sweeps: int = 0, opts: Optional[hjb_solve_opts] = None, stream=None,
                      device: bool = False, allow_noconv: bool = False) -> dict:
    """v_out: torch CUDA tensor of N float32 (HJB_F32) or float64 (HJB_F64)."""
    P = _as_problem(fine, device)
    _check_out(v_out, P.N, precision)
    st = hjb_stats()
    rc = lib.hjb_solve_patches(P.ref, patches.h, int(precision), float(tol), int(max_sweeps),
                               v_out.data_ptr(), None if opts is None else C.byref(opts),
                               C.byref(st), _stream(stream))
    _check(rc, "hjb_solve_patches", (HJB_OK, HJB_ENOCONV) if allow_noconv else (HJB_OK,))
    return st.as_dict()


def hjb_solve_global(fine, precision: int, v_out, tol: float = 0.0, max_sweeps: int = 0,
                     opts: Optional[hjb_solve_opts] = None, stream=None, device: bool = False,
                     allow_noconv: bool = False) -> dict:
    P = _as_problem(fine, device)
    _check_out(v_out, P.N, precision)
    st = hjb_stats()
    rc = lib.hjb_solve_global(P.ref, int(precision), float(tol), int(max_sweeps), v_out.data_ptr(),
                              None if opts is None else C.byref(opts), C.byref(st), _stream(stream))
    _check(rc, "hjb_solve_global", (HJB_OK, HJB_ENOCONV) if allow_noconv else (HJB_OK,))
    return st.as_dict()


def hjb_solve_global_noalloc(fine, precision: int, v_out, tol: float = 0.0, max_sweeps: int = 0,
                             stream=None, allow_noconv: bool = False) -> dict:
    """The plain global solve (HJB_SCHED_JACOBI) with no device allocation:
    `fine` must hold device inputs (Problem(..., device=True))."""
    P = _as_problem(fine)
    _check_out(v_out, P.N, precision)
    st = hjb_stats()
    rc = lib.hjb_solve_global_noalloc(P.ref, int(precision), float(tol), int(max_sweeps),
                                      v_out.data_ptr(), C.byref(st), _stream(stream))
    _check(rc, "hjb_solve_global_noalloc", (HJB_OK, HJB_ENOCONV) if allow_noconv else (HJB_OK,))
    return st.as_dict()


def _check_out(v_out, N, precision):
    import torch
    want = torch.float32 if precision == HJB_F32 else torch.float64
    if not (v_out.is_cuda and v_out.dtype == want and v_out.numel() == N and v_out.is_contiguous()):
        raise ValueError(f"v_out must be a contiguous CUDA tensor of {N} {want}")


# ---------------------------------------------------------------- batch


class Batch:
    def __init__(self, fines: Sequence, coarses: Sequence, precision: int = HJB_F32,
                 tol: float = 0.0, max_sweeps: int = 0, opts: Optional[hjb_solve_opts] = None,
                 stream=None, device: bool = False, prepare_bytes: int = 0):
        self.fines = [_as_problem(f, device) for f in fines]
        self.coarses = [_as_problem(c, device) for c in coarses]
        n = len(self.fines)
        F = (C.POINTER(hjb_problem) * n)(*[C.pointer(p.s) for p in self.fines])
        Cc = (C.POINTER(hjb_problem) * n)(*[C.pointer(p.s) for p in self.coarses])
        bo = hjb_batch_opts()
        bo.precision = int(precision)
        bo.tol = float(tol)
        bo.max_sweeps = int(max_sweeps)
        bo.prepare_bytes = int(prepare_bytes)
        if opts is not None:
            bo.solve = opts
        self.precision = precision
        self.stream = _stream(stream)
        h = C.c_void_p()
        _check(lib.hjb_batch_create(F, Cc, n, C.byref(bo), self.stream, C.byref(h)),
               "hjb_batch_create")
        self.h = h.value

    def run(self) -> dict:
        st = hjb_stats()
        _check(lib.hjb_batch_run(self.h, self.stream, C.byref(st)), "hjb_batch_run")
        return st.as_dict()

    def result(self, i: int, out=None):
        N = self.fines[i].N
        if out is None:
            out = np.empty(N, dtype=np.float32 if self.precision == HJB_F32 else np.float64)
        st = hjb_stats()
        mem = HJB_MEM_HOST if isinstance(out, np.ndarray) else HJB_MEM_DEVICE
        _check(lib.hjb_batch_result(self.h, int(i), _ptr(out), mem, C.byref(st)), "hjb_batch_result")
        return out, st.as_dict()

    def free(self):
        if getattr(self, "h", None) and lib is not None:
            lib.hjb_batch_free(self.h)
        self.h = None

    def __del__(self):
        self.free()


def hjb_batch_create(fines, coarses, precision=HJB_F32, tol=0.0, max_sweeps=0, opts=None,
                     stream=None, device=False, prepare_bytes=0) -> Batch:
    return Batch(fines, coarses, precision, tol, max_sweeps, opts, stream, device, prepare_bytes)


def hjb_batch_run(b: Batch) -> dict:
    return b.run()


def hjb_batch_result(b: Batch, i: int, out=None):
    return b.result(i, out)


def hjb_batch_free(b: Batch) -> None:
    b.free()


# ---------------------------------------------------------------- serving


class Server:
    def __init__(self, hbm_budget: int, precision: int = HJB_F32, tol: float = 0.0,
                 max_sweeps: int = 0, opts: Optional[hjb_solve_opts] = None, stream=None):
        so = hjb_server_opts()
        so.precision = int(precision)
        so.tol = float(tol)
        so.max_sweeps = int(max_sweeps)
        if opts is not None:
            so.solve = opts
        self.precision = precision
        self.sizes = {}
        h = C.c_void_p()
        _check(lib.hjb_server_create(int(hbm_budget), C.byref(so), _stream(stream), C.byref(h)),
               "hjb_server_create")
        self.h = h.value

    def submit(self, fine, coarse) -> int:
        F, Cc = _as_problem(fine), _as_problem(coarse)
        t = C.c_uint64()
        _check(lib.hjb_server_submit(self.h, F.ref, Cc.ref, C.byref(t)), "hjb_server_submit")
        self.sizes[t.value] = F.N
        return t.value

    def step(self, rounds: int = 6):
        live, queued = C.c_int32(), C.c_int32()
        _check(lib.hjb_server_step(self.h, int(rounds), C.byref(live), C.byref(queued)),
               "hjb_server_step")
        return live.value, queued.value

    def poll(self, ticket: int, out=None):
        """(None, None) while the request runs; then (values, stats)."""
        N = self.sizes[ticket]
        if out is None:
            out = np.empty(N, dtype=np.float32 if self.precision == HJB_F32 else np.float64)
        st = hjb_stats()
        mem = HJB_MEM_HOST if isinstance(out, np.ndarray) else HJB_MEM_DEVICE
        rc = lib.hjb_server_poll(self.h, C.c_uint64(ticket), _ptr(out), mem, C.byref(st))
        if rc == HJB_EAGAIN:
            return None, None
        # collected: a result, or the error of a request that failed
        del self.sizes[ticket]
        _check(rc, "hjb_server_poll", (HJB_OK, HJB_ENOCONV))
        return out, st.as_dict()

    def free(self):
        if getattr(self, "h", None) and lib is not None:
            lib.hjb_server_free(self.h)
        self.h = None

    def __del__(self):
        self.free()


def hjb_server_create(hbm_budget, precision=HJB_F32, tol=0.0, max_sweeps=0, opts=None,
                      stream=None) -> Server:
    return Server(hbm_budget, precision, tol, max_sweeps, opts, stream)


def hjb_server_submit(s: Server, fine, coarse) -> int:
    return s.submit(fine, coarse)


def hjb_server_step(s: Server, rounds: int = 6):
    return s.step(rounds)


def hjb_server_poll(s: Server, ticket: int, out=None):
    return s.poll(ticket, out)


def hjb_server_free(s: Server) -> None:
    s.free()


def patchy_solve(fine, coarse, precision: int = HJB_F32, tol: float = 0.0, stream=None,
                 device: bool = False, opts: Optional[hjb_solve_opts] = None):
    """The three calls of the Patchy Algorithm in a row; returns
    (v tensor, labels handle, stats per step)."""
    import torch
    Fp = _as_problem(fine, device)
    Cp = _as_problem(coarse, device)
    ch = hjb_coarse_solve(Cp, 0.0, 0, stream)
    ph = hjb_build_patches(Fp, ch, stream)
    ch.free()
    v = torch.empty(Fp.N, dtype=torch.float32 if precision == HJB_F32 else torch.float64,
                    device="cuda")
    st = hjb_solve_patches(Fp, ph, precision, v, tol, 0, opts, stream)
    return v, ph, dict(build=ph.stats, solve=st)
