"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Bars: labels, feedback and FP64 values bit-exact (every FP64 kernel evaluates
the same IEEE operations in the same order as the oracle, and every fair
schedule of the monotone iteration stops on the same fixed point); FP32
values within 1e-5 of the FP64 oracle in the sup norm.
"""
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


def test_global_fp64_exact_config1(H, orc, pr):
    """Eikonal 101^2, FP64: the tiled GPU schedule and the plain GPU Jacobi
    both stop on the oracle's fixed point, bit for bit."""
    P = pr.config1()
    ref, _ = orc.solve_global(P)
    v = _zeros(P.N, True)
    st = H.hjb_solve_global(P, H.HJB_F64, v)
    assert np.array_equal(_np(v), ref)
    assert st["updates"] > 0 and st["rounds"] > 0
    vj = _zeros(P.N, True)
    H.hjb_solve_global(P, H.HJB_F64, vj, opts=H.make_opts(schedule=H.HJB_SCHED_JACOBI))
    assert np.array_equal(_np(vj), ref)


def test_global_fp32_config1(H, orc, pr):
    P = pr.eikonal_2d(101, 32, 0.1, fp32=True)
    ref, _ = orc.solve_global(P)
    for sched in (H.HJB_SCHED_TILED, H.HJB_SCHED_JACOBI):
        v = _zeros(P.N, False)
        H.hjb_solve_global(P, H.HJB_F32, v, opts=H.make_opts(schedule=sched))
        assert np.abs(_np(v) - ref).max() <= 1e-5


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_coarse_solve_exact_2d(H, orc, pr, seed):
    _, c = pr.config2(seed, n=129, nc_coarse=65)
    ref, _ = orc.solve_global(c)
    ch = H.hjb_coarse_solve(c)
    assert np.array_equal(ch.values(), ref)


def test_coarse_solve_exact_3d(H, orc, pr):
    _, c = pr.config3(0, n=65, nc_coarse=33)
    ref, _ = orc.solve_global(c)
    ch = H.hjb_coarse_solve(c)
    assert np.array_equal(ch.values(), ref)


def _build_compare(H, orc, f, c):
    vc, _ = orc.solve_global(c)
    u0 = orc.prolong(c, vc, f)
    fb = orc.feedback(f, u0)
    lab, un = orc.labels(f, fb, want_unreached=True)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    assert np.array_equal(ph.u0(), u0)
    assert np.array_equal(ph.feedback(), fb)
    assert np.array_equal(ph.labels(), lab)
    assert ph.stats["unreached"] == un
    assert lab.min() >= 0
    return ph, lab


def test_build_patches_label_fill(H, orc, pr):
    """Remark 3.1 fill on the GPU: a block of standing nodes (speed 0) that no
    colour reaches, on a grid that is not a multiple of the tile sides."""
    n = 133
    f = pr.line_target_2d(n, 16, strips=3)
    c = pr.line_target_2d(17, 16, strips=3)
    speed = f.speed.reshape(n, n).copy()
    speed[40:80, 90:110] = 0.0
    f.speed = speed.ravel()
    ph, lab = _build_compare(H, orc, f, c)
    assert ph.stats["unreached"] >= 40 * 20


def test_build_patches_rotating_drift(H, orc, pr):
    """A serving request whose rotating drift makes near-closed loops of the
    frozen feedback: the discounted colour transport must settle, bit for bit
    with the oracle."""
    s = np.random.SeedSequence(0).spawn(49)[48]
    f, c = pr.batched_problem(s, 48, (167, 167))
    _build_compare(H, orc, f, c)


@pytest.mark.parametrize("n,nc,R", [(129, 17, 16), (257, 33, 16), (130, 17, 5)])
def test_build_patches_exact_2d(H, orc, pr, n, nc, R):
    """Steps 2 and 3.1 on ragged grids (not multiples of any tile side)."""
    f, c = pr.variable_speed_2d(0, n, nc, 32, R, 0.1, True)
    _build_compare(H, orc, f, c)


def test_build_patches_exact_3d(H, orc, pr):
    f, c = pr.variable_speed_3d(1, 41, 11, 98, 4, 4, 0.25, True)
    _build_compare(H, orc, f, c)


def test_build_patches_exact_drift(H, orc, pr):
    f, c = pr.variable_speed_2d(5, 131, 17, 24, 7, 0.1, True, drift_sign=-1)
    _build_compare(H, orc, f, c)


@pytest.mark.parametrize("case", ["2d", "2d_drift", "3d"])
def test_solve_patches_parity(H, orc, pr, case):
    """Steps 3.2 and 4: FP64 bit-exact, FP32 within 1e-5."""
    if case == "2d":
        f, c = pr.variable_speed_2d(2, 193, 17, 32, 16, 0.1, True)
    elif case == "2d_drift":
        f, c = pr.variable_speed_2d(3, 150, 17, 20, 9, 0.1, True, drift_sign=1)
    else:
        f, c = pr.variable_speed_3d(0, 37, 11, 98, 4, 4, 0.25, True)
    out = orc.patchy(f, c)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    assert np.array_equal(ph.labels(), out["labels"])
    v64 = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, v64)
    assert np.array_equal(_np(v64), out["v"])
    v32 = _zeros(f.N, False)
    st = H.hjb_solve_patches(f, ph, H.HJB_F32, v32)
    assert np.abs(_np(v32) - out["v"]).max() <= 1e-5
    assert st["updates"] == st["node_updates"] * f.n_controls
    # the asynchronous schedule (one persistent launch, device work queue)
    # reaches the same fixed point bit for bit
    a64 = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, a64, opts=H.make_opts(schedule=H.HJB_SCHED_ASYNC))
    assert np.array_equal(_np(a64), out["v"])
    a32 = _zeros(f.N, False)
    v32e = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, v32e, 0.0)
    H.hjb_solve_patches(f, ph, H.HJB_F32, a32, 0.0, opts=H.make_opts(schedule=H.HJB_SCHED_ASYNC))
    assert np.array_equal(_np(a32), _np(v32e))


def test_async_schedule_rejects_cap(H, pr):
    f, c = pr.variable_speed_2d(1, 65, 17, 16, 4, 0.1, True)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    v = _zeros(f.N, False)
    with pytest.raises(H.HjbError) as e:
        H.hjb_solve_patches(f, ph, H.HJB_F32, v, 0.0, 10, H.make_opts(schedule=H.HJB_SCHED_ASYNC))
    assert e.value.status == H.HJB_EINVAL


def test_fp32_schedules_bitwise_equal(H, pr):
    """Tile shape, in-tile sweep count, polling and graph replay change the
    order of the (monotone) updates but not the FP32 fixed point."""
    f, c = pr.variable_speed_2d(4, 201, 17, 32, 8, 0.1, True)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    import torch
    outs = []
    stream = torch.cuda.Stream()  # graphs cannot be captured on the null stream
    with torch.cuda.stream(stream):
        for tile, K, rpp, graph, sched in [
                ((64, 16, 1), 48, 6, False, H.HJB_SCHED_TILED),
                ((32, 32, 1), 8, 1, False, H.HJB_SCHED_TILED),
                ((64, 8, 1), 200, 12, True, H.HJB_SCHED_TILED),
                ((32, 16, 1), 1, 6, True, H.HJB_SCHED_TILED),
                ((16, 16, 1), 3, 0, False, H.HJB_SCHED_ASYNC),
                ((32, 8, 1), 64, 0, False, H.HJB_SCHED_ASYNC)]:
            v = _zeros(f.N, False)
            H.hjb_solve_patches(f, ph, H.HJB_F32, v,
                                opts=H.make_opts(tile=tile, inner_sweeps=K, rounds_per_poll=rpp,
                                                 use_graph=graph, schedule=sched))
            outs.append(_np(v))
    torch.cuda.synchronize()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_fp32_schedules_bitwise_equal_3d(H, pr):
    f, c = pr.variable_speed_3d(1, 45, 11, 98, 2, 4, 0.25, True)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    outs = []
    for tile, K, sched in [((16, 8, 8), 32, H.HJB_SCHED_TILED), ((8, 8, 8), 3, H.HJB_SCHED_TILED),
                           ((32, 8, 4), 100, H.HJB_SCHED_TILED), ((8, 8, 8), 4, H.HJB_SCHED_ASYNC)]:
        v = _zeros(f.N, False)
        H.hjb_solve_patches(f, ph, H.HJB_F32, v,
                            opts=H.make_opts(tile=tile, inner_sweeps=K, schedule=sched))
        outs.append(_np(v))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_patch_subset_independence(H, pr):
    """Solving a subset of the patches gives the same bits on them as the
    full run (patches exchange nothing during Step 3.2): the basis for
    sharding patches across devices."""
    f, c = pr.variable_speed_2d(6, 257, 17, 32, 16, 0.1, True)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    lab = ph.labels()
    full = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, full)
    sel = np.zeros(16, dtype=np.uint8)
    sel[[1, 5, 6, 11]] = 1
    part = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, part, opts=H.make_opts(patch_select=sel))
    m = np.isin(lab, [1, 5, 6, 11]) & (f.target_part < 0)
    assert np.array_equal(_np(part)[m], _np(full)[m])
    other = (~np.isin(lab, [1, 5, 6, 11])) & (f.target_part < 0)
    assert np.all(_np(part)[other] == 1.0)


def test_single_patch_equals_global(H, pr):
    f, c = pr.variable_speed_2d(1, 129, 17, 32, 1, 0.1, True)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    a, b = _zeros(f.N, False), _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, a)
    H.hjb_solve_global(f, H.HJB_F32, b)
    assert np.array_equal(_np(a), _np(b))


def test_round_cap_gives_upper_bound(H, orc, pr):
    """HJB_ENOCONV when max_sweeps is hit; the iterate is >= the fixed point."""
    P = pr.eikonal_2d(121, 32, 0.1)
    ref, _ = orc.solve_global(P)
    v = _zeros(P.N, True)
    st = H.hjb_solve_global(P, H.HJB_F64, v, max_sweeps=2, allow_noconv=True)
    assert st["status"] == H.HJB_ENOCONV
    assert np.all(_np(v) >= ref) and np.any(_np(v) > ref)
    vj = _zeros(P.N, True)
    st = H.hjb_solve_global(P, H.HJB_F64, vj, max_sweeps=3, allow_noconv=True,
                            opts=H.make_opts(schedule=H.HJB_SCHED_JACOBI))
    assert st["status"] == H.HJB_ENOCONV and np.all(_np(vj) >= ref)


def test_degenerate_grids(H, orc, pr):
    """Smallest grid (2x2), every node a target, and a grid the target does
    not reach under the state constraint."""
    P = pr.eikonal_2d(2, 8, 1.0, h=0.5)  # 2x2 grid with one target corner
    P.target_part = np.array([0, -1, -1, -1], dtype=np.int16)
    ref, _ = orc.solve_global(P)
    v = _zeros(P.N, True)
    H.hjb_solve_global(P, H.HJB_F64, v)
    assert np.array_equal(_np(v), ref)
    P = pr.eikonal_2d(9, 8, 5.0)  # every node inside the target
    v = _zeros(P.N, True)
    H.hjb_solve_global(P, H.HJB_F64, v)
    assert np.all(_np(v) == 0.0)
    P = pr.eikonal_2d(33, 8, 0.1)
    P.speed = np.zeros(P.N)  # nobody moves: only the target has a finite time
    ref, _ = orc.solve_global(P)
    v = _zeros(P.N, True)
    H.hjb_solve_global(P, H.HJB_F64, v)
    assert np.array_equal(_np(v), ref)
    assert np.all(_np(v)[P.target_part < 0] == 1.0)


def test_tolerance_stop(H, orc, pr):
    """tol > 0 stops early; the result stays an upper bound within a small
    multiple of tol / (1 - beta) of the fixed point."""
    f, c = pr.variable_speed_2d(0, 129, 17, 32, 4, 0.1, True)
    ref, _ = orc.solve_global(f)
    v = _zeros(f.N, False)
    st = H.hjb_solve_global(f, H.HJB_F32, v, tol=1e-5)
    e = _np(v) - ref
    assert e.min() >= -1e-5 and e.max() <= 1e-5 / (1 - f.beta)
    assert st["status"] == H.HJB_OK


def test_device_resident_inputs(H, orc, pr):
    """mem = HJB_MEM_DEVICE: the same results from torch-resident inputs."""
    f, c = pr.variable_speed_2d(1, 97, 17, 16, 4, 0.1, True, drift_sign=1)
    out = orc.patchy(f, c)
    ch = H.hjb_coarse_solve(c, device=True)
    ph = H.hjb_build_patches(f, ch, device=True)
    assert np.array_equal(ph.labels(), out["labels"])
    v = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, v, device=True)
    assert np.array_equal(_np(v), out["v"])


@pytest.mark.parametrize("case", ["2d", "2d_drift"])
def test_control_slices_bitwise_equal(H, orc, pr, case):
    """Workgroups with more threads than tile nodes split each node's
    controls over 2 or 4 slices; the minimum is exact, so FP64 stays
    bit-exact against the oracle and FP32 keeps the bits of one slice."""
    if case == "2d":
        f, c = pr.variable_speed_2d(5, 131, 17, 32, 8, 0.1, True)
    else:
        f, c = pr.variable_speed_2d(6, 97, 17, 20, 6, 0.1, True, drift_sign=-1)
    out = orc.patchy(f, c)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    ref32 = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, ref32)
    for tile, nt, K, sched in [((32, 8, 1), 512, 8, H.HJB_SCHED_TILED),
                               ((32, 8, 1), 1024, 12, H.HJB_SCHED_TILED),
                               ((16, 16, 1), 512, 3, H.HJB_SCHED_TILED),
                               ((16, 16, 1), 1024, 8, H.HJB_SCHED_ASYNC),
                               ((32, 16, 1), 1024, 16, H.HJB_SCHED_TILED)]:
        o = H.make_opts(tile=tile, threads=nt, inner_sweeps=K, schedule=sched)
        v64 = _zeros(f.N, True)
        st = H.hjb_solve_patches(f, ph, H.HJB_F64, v64, opts=o)
        assert st["threads"] == nt
        assert np.array_equal(_np(v64), out["v"]), (tile, nt)
        v32 = _zeros(f.N, False)
        H.hjb_solve_patches(f, ph, H.HJB_F32, v32, opts=o)
        assert np.array_equal(_np(v32), _np(ref32)), (tile, nt)
    # the global solve (and so the coarse solve) with slices is the exact
    # fixed point of the oracle's Jacobi iteration
    g = _zeros(c.N, True)
    H.hjb_solve_global(c, H.HJB_F64, g, opts=H.make_opts(tile=(16, 16, 1), threads=1024,
                                                          inner_sweeps=8))
    assert np.array_equal(_np(g), orc.solve_global(c)[0])
