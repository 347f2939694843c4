"""Obstacles (Section 4.5) and exclusion of unreachable regions after Step 1
(Section 4.6) through the C ABI: coarse values, U^(0), feedback and labels
bit-exact with the oracle, FP64 values bit-exact, FP32 within 1e-5."""
import dataclasses

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


def _box3d(pr):
    f, c = pr.variable_speed_3d(1, 37, 13, 98, 2, 2, 0.3, True)
    def box(P):
        X, Y, Z = P.coords()
        return ((np.abs(X - 0.55) < 0.15) & (np.abs(Y) < 0.5) & (np.abs(Z) < 0.5)).ravel()
    return pr.with_obstacles(f, box(f)), pr.with_obstacles(c, box(c))


def _ring2d(pr):
    f0 = pr.eikonal_2d(97, 32, 0.1, 4, fp32=True)
    c0 = pr.eikonal_2d(25, 32, 0.1, 4)
    def ring(P):
        X, Y = P.coords()
        r = np.hypot(X - 0.5, Y - 0.5)
        return ((r >= 0.25) & (r <= 0.4)).ravel()
    return pr.with_obstacles(f0, ring(f0)), pr.with_obstacles(c0, ring(c0))


def _case(pr, case):
    if case == "disc_rect":
        return pr.eikonal_obstacles_2d(161, 32, 8, fp32=True), None
    if case == "box3d":
        return _box3d(pr), None
    if case == "zermelo_exclude":
        z = pr.zermelo_2d(101, 32, c=0.6, w=(0.9, 0.0), r=0.2, fp32=True)
        zc = pr.zermelo_2d(26, 32, c=0.6, w=(0.9, 0.0), r=0.2)
        return (z, zc), 1.0
    return _ring2d(pr), 1.0


@pytest.mark.parametrize("case", ["disc_rect", "box3d", "zermelo_exclude", "ring_exclude"])
def test_obstacle_parity(H, orc, pr, case):
    (f, c), theta = _case(pr, case)
    print(f"[obst] {case}", flush=True)
    out = orc.patchy(f, c, exclude_at=theta)
    ch = H.hjb_coarse_solve(c)
    assert np.array_equal(ch.values(), out["v_coarse"])
    ph = H.hjb_build_patches(f, ch, exclude_at=theta)
    assert np.array_equal(ph.u0(), out["u0"])
    assert np.array_equal(ph.feedback(), out["feedback"])
    assert np.array_equal(ph.labels(), out["labels"])
    assert ph.stats["excluded"] == out["excluded"]
    v64 = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, v64)
    assert np.array_equal(_np(v64), out["v"])
    v32 = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, v32)
    assert np.abs(_np(v32) - out["v"]).max() <= 1e-5
    # the Dirichlet patch data never reach into an obstacle
    fe = dataclasses.replace(f, target_part=out["target_part"])
    ref_d, _ = orc.solve_patches_ex(fe, out["labels"], u0=out["u0"])
    d64 = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, d64, opts=H.make_opts(patch_bc=H.HJB_BC_DIRICHLET))
    assert np.array_equal(_np(d64), ref_d)


def test_obstacle_global_solves(H, orc, pr):
    f, _ = pr.eikonal_obstacles_2d(129, 32, 8)
    ref, _ = orc.solve_global(f)
    for sched in (H.HJB_SCHED_TILED, H.HJB_SCHED_JACOBI, H.HJB_SCHED_ASYNC):
        v = _zeros(f.N, True)
        H.hjb_solve_global(f, H.HJB_F64, v, opts=H.make_opts(schedule=sched))
        assert np.array_equal(_np(v), ref), sched


def test_obstacle_batch_equals_alone(H, pr):
    probs = [pr.eikonal_obstacles_2d(129, 32, 8, fp32=True), _box3d(pr),
             pr.variable_speed_2d(3, 97, 17, 32, 6, 0.1, True)]
    alone = []
    for f, c in probs:
        ch = H.hjb_coarse_solve(c)
        ph = H.hjb_build_patches(f, ch)
        v = _zeros(f.N, False)
        H.hjb_solve_patches(f, ph, H.HJB_F32, v)
        alone.append(v.cpu().numpy())
    b = H.hjb_batch_create([f for f, _ in probs], [c for _, c in probs], H.HJB_F32)
    H.hjb_batch_run(b)
    for i in range(len(probs)):
        got, _ = H.hjb_batch_result(b, i)
        assert np.array_equal(got, alone[i]), i


def test_exclusion_rejections(H, pr):
    f, c = pr.variable_speed_2d(1, 65, 17, 16, 4, 0.1, True)
    ch = H.hjb_coarse_solve(c)
    for theta in (-0.5, 1.5, float("nan")):
        with pytest.raises(H.HjbError) as e:
            H.hjb_build_patches(f, ch, exclude_at=theta)
        assert e.value.status == H.HJB_EINVAL
    P = dataclasses.replace(f, target_part=np.where(f.target_part < 0, -3, f.target_part)
                            .astype(np.int16))
    with pytest.raises(H.HjbError) as e:
        H.hjb_build_patches(P, ch)
    assert e.value.status == H.HJB_EINVAL
