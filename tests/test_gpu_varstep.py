"""The paper's variable step h_i (Section 2.1) through the C ABI: per-node
beta_i in the scheme and in the colour transport.  Coarse values, U^(0),
feedback and labels bit-exact with the oracle, FP64 values bit-exact, FP32
within 1e-5; device-resident inputs; batches equal solves alone."""
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
    if case == "fan2d":
        return pr.fan_2d(129, 32, 16, fp32=True), pr.fan_2d(33, 32, 16)
    if case == "fan3d":
        return pr.fan_3d(33, 98, 8, fp32=True), pr.fan_3d(17, 98, 8)
    f, c = pr.variable_speed_2d(5, 97, 17, 32, 8, 0.1, True)
    return pr.unit_reach(f, True), pr.unit_reach(c, False)


@pytest.mark.parametrize("case", ["fan2d", "fan3d", "varspeed_unit"])
def test_varstep_parity(H, orc, pr, case):
    f, c = _case(pr, case)
    print(f"[varstep] {case}", flush=True)
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
    # the global solves (tiled and plain Jacobi) use the same per-node beta
    ref, _ = orc.solve_global(f)
    for sched in (H.HJB_SCHED_TILED, H.HJB_SCHED_JACOBI):
        g = _zeros(f.N, True)
        H.hjb_solve_global(f, H.HJB_F64, g, opts=H.make_opts(schedule=sched))
        assert np.array_equal(_np(g), ref), sched


def test_varstep_with_addons(H, orc, pr):
    f, c = pr.fan_2d(97, 32, 8), pr.fan_2d(25, 32, 8)
    out = orc.patchy(f, c)
    ref, _ = orc.solve_patches_ex(f, out["labels"], out["feedback"], 4.0, out["u0"])
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    v64 = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, v64,
                        opts=H.make_opts(control_cone=4.0, patch_bc=H.HJB_BC_DIRICHLET,
                                         order_window=4.0))
    assert np.array_equal(_np(v64), ref)


def test_varstep_batch_equals_alone(H, pr):
    probs = [_case(pr, "fan2d"), _case(pr, "varspeed_unit"),
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


def test_varstep_rejections(H, pr):
    f = pr.fan_2d(33, 16, 4)
    for bad in (1.0, -0.1, float("nan")):
        bn = f.beta_node.copy()
        bn[7] = bad
        P = dataclasses.replace(f, beta_node=bn)
        for device in (False, True):
            with pytest.raises(H.HjbError) as e:
                H.hjb_coarse_solve(P, device=device)
            assert e.value.status == H.HJB_EINVAL
