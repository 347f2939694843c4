"""Tabulated dynamics (foot-point displacement and beta per control and
node) through the C ABI: the paper's Zermelo (Table test2d), Brockett's
integrator (Table test3d) and Lunar landing (Section 4.6) with the step rule
of Section 2.1.  Coarse values, U^(0), feedback and labels bit-exact with
the oracle, FP64 values bit-exact, FP32 within 1e-5."""
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


def _case(pr, case):
    if case == "zermelo":
        return pr.zermelo_paper_2d(129, 32, 16, fp32=True), pr.zermelo_paper_2d(33, 32, 16)
    if case == "brockett":
        return pr.brockett_3d(33, 8, fp32=True), pr.brockett_3d(17, 8)
    return pr.lunar_landing_2d(81, 0.12, 4, fp32=True), pr.lunar_landing_2d(41, 0.12, 4)


@pytest.mark.parametrize("case", ["zermelo", "brockett", "lunar"])
def test_tabulated_parity(H, orc, pr, case):
    f, c = _case(pr, case)
    print(f"[tab] {case}", flush=True)
    out = orc.patchy(f, c)
    for device in (False, True):
        ch = H.hjb_coarse_solve(c, device=device)
        assert np.array_equal(ch.values(), out["v_coarse"])
        ph = H.hjb_build_patches(f, ch, device=device)
        assert np.array_equal(ph.u0(), out["u0"])
        assert np.array_equal(ph.feedback(), out["feedback"])
        assert np.array_equal(ph.labels(), out["labels"])
        v64 = _zeros(f.N, True)
        H.hjb_solve_patches(f, ph, H.HJB_F64, v64, device=device)
        assert np.array_equal(_np(v64), out["v"])
        v32 = _zeros(f.N, False)
        H.hjb_solve_patches(f, ph, H.HJB_F32, v32, device=device)
        assert np.abs(_np(v32) - out["v"]).max() <= 1e-5
    ref, _ = orc.solve_global(f)
    for sched in (H.HJB_SCHED_TILED, H.HJB_SCHED_JACOBI):
        g = _zeros(f.N, True)
        H.hjb_solve_global(f, H.HJB_F64, g, opts=H.make_opts(schedule=sched))
        assert np.array_equal(_np(g), ref), sched


def test_table_equals_model(H, pr):
    """A table holding s (c a + w) gives the model's bits on the GPU too."""
    f, _ = pr.variable_speed_2d(3, 65, 17, 20, 4, 0.1, False, drift_sign=1)
    foot = np.zeros((f.n_controls, f.N, 2))
    for k in range(f.n_controls):
        for d in range(2):
            g = f.speed * f.controls[k, d]
            g = g + f.drift[:, d]
            foot[k, :, d] = f.step[d] * g
    a = _zeros(f.N, True)
    H.hjb_solve_global(f, H.HJB_F64, a)
    b = _zeros(f.N, True)
    H.hjb_solve_global(dataclasses.replace(f, foot=foot), H.HJB_F64, b)
    assert np.array_equal(_np(a), _np(b))


def test_tabulated_with_addons(H, orc, pr):
    f, c = pr.zermelo_paper_2d(97, 32, 8), pr.zermelo_paper_2d(25, 32, 8)
    out = orc.patchy(f, c)
    ref, _ = orc.solve_patches_ex(f, out["labels"], u0=out["u0"])
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    v64 = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, v64,
                        opts=H.make_opts(patch_bc=H.HJB_BC_DIRICHLET, order_window=3.0))
    assert np.array_equal(_np(v64), ref)


def test_tabulated_rejections(H, pr):
    f, c = pr.zermelo_paper_2d(33, 16, 4), pr.zermelo_paper_2d(17, 16, 4)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    v = _zeros(f.N, False)
    for o in (H.make_opts(schedule=H.HJB_SCHED_ASYNC), H.make_opts(control_cone=4.0),
              H.make_opts(tile=(64, 16, 1), threads=256)):
        with pytest.raises(H.HjbError) as e:
            H.hjb_solve_patches(f, ph, H.HJB_F32, v, opts=o)
        assert e.value.status == H.HJB_EINVAL
    with pytest.raises(H.HjbError) as e:
        H.hjb_batch_create([f], [c])
    assert e.value.status == H.HJB_EINVAL
    far = f.foot.copy()
    far[3, 10, 0] = 2.5
    nobeta = dataclasses.replace(f, foot=None)
    for bad in (dataclasses.replace(f, foot=far), nobeta):
        for device in (False, True):
            with pytest.raises(H.HjbError) as e:
                H.hjb_coarse_solve(bad, device=device)
            assert e.value.status == H.HJB_EINVAL
