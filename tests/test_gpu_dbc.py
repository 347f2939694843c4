"""Dirichlet patch boundary data (eq. dbc): in Step 3.2 the nodes of other
patches hold U^(0) of Step 2 instead of the ghost value 1.  Parity of the
HIP path with the oracle's solve_patches_ex: FP64 bit-exact (the iteration
still starts above the fixed point and decreases monotonically), FP32 within
1e-5; batches and the server give each problem the bits of its solve alone.
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


def _case(pr, case):
    if case == "c2_257":
        # the headline generator at 257^2 / 17^2: patches that straddle
        # tiles, nodes of other patches as Dirichlet data next to every
        # patch
        return pr.config2(0, 257, pr.coarse_size_2d(257))
    if case == "2d":
        return pr.variable_speed_2d(2, 193, 17, 32, 16, 0.1, True)
    if case == "2d_drift":
        return pr.variable_speed_2d(3, 150, 17, 20, 9, 0.1, True, drift_sign=1)
    return pr.variable_speed_3d(0, 37, 11, 98, 4, 4, 0.25, True)


@pytest.mark.parametrize("case", ["2d", "2d_drift", "3d", "c2_257"])
def test_dbc_solve_parity(H, orc, pr, case):
    f, c = _case(pr, case)
    out = orc.patchy(f, c)
    ref, _ = orc.solve_patches_ex(f, out["labels"], u0=out["u0"])
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    assert np.array_equal(ph.u0(), out["u0"])
    assert np.array_equal(ph.labels(), out["labels"])
    print(f"[dbc] {case} tiled / async", flush=True)
    o = H.make_opts(patch_bc=H.HJB_BC_DIRICHLET)
    v64 = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, v64, opts=o)
    assert np.array_equal(_np(v64), ref)
    a64 = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, a64,
                        opts=H.make_opts(patch_bc=H.HJB_BC_DIRICHLET,
                                         schedule=H.HJB_SCHED_ASYNC))
    assert np.array_equal(_np(a64), ref)
    v32 = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, v32, opts=o)
    assert np.abs(_np(v32) - ref).max() <= 1e-5
    # the data differ from the ghost value: the result differs from the
    # state-constraint solve
    assert not np.array_equal(ref, out["v"])


def test_dbc_with_control_cone(H, orc, pr):
    """Eq. dbc and add-on AO3 together, as in the paper's add-on runs."""
    f, c = pr.variable_speed_2d(6, 161, 17, 32, 8, 0.1, True)
    out = orc.patchy(f, c)
    ref, _ = orc.solve_patches_ex(f, out["labels"], out["feedback"], 4.0, out["u0"])
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    o = H.make_opts(patch_bc=H.HJB_BC_DIRICHLET, control_cone=4.0)
    v64 = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, v64, opts=o)
    assert np.array_equal(_np(v64), ref)
    v32 = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, v32, opts=o)
    assert np.abs(_np(v32) - ref).max() <= 1e-5


def test_dbc_batch_and_server_equal_alone(H, pr):
    probs = [pr.variable_speed_2d(7, 97, 17, 24, 6, 0.1, True),
             pr.variable_speed_2d(8, 130, 17, 32, 12, 0.1, True, drift_sign=-1),
             pr.variable_speed_3d(3, 29, 9, 98, 2, 4, 0.3, True, "b3d")]
    o = H.make_opts(patch_bc=H.HJB_BC_DIRICHLET)
    alone = []
    for f, c in probs:
        ch = H.hjb_coarse_solve(c)
        ph = H.hjb_build_patches(f, ch)
        v = _zeros(f.N, False)
        H.hjb_solve_patches(f, ph, H.HJB_F32, v, opts=o)
        alone.append(v.cpu().numpy())
    b = H.hjb_batch_create([f for f, _ in probs], [c for _, c in probs], H.HJB_F32, opts=o)
    H.hjb_batch_run(b)
    for i in range(len(probs)):
        got, _ = H.hjb_batch_result(b, i)
        assert np.array_equal(got, alone[i]), i
    S = H.hjb_server_create(2 << 30, H.HJB_F32, opts=o)
    tickets = [S.submit(f, c) for f, c in probs]
    done = {}
    for _ in range(20000):
        S.step(4)
        for i, t in enumerate(tickets):
            if i not in done:
                v, st = S.poll(t)
                if v is not None:
                    done[i] = v
        if len(done) == len(probs):
            break
    for i in range(len(probs)):
        assert np.array_equal(done[i], alone[i]), i


def test_dbc_rejections(H, pr):
    f, c = pr.variable_speed_2d(1, 65, 17, 16, 4, 0.1, True)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    v = _zeros(f.N, False)
    with pytest.raises(H.HjbError) as e:
        H.hjb_solve_patches(f, ph, H.HJB_F32, v, opts=H.make_opts(patch_bc=7))
    assert e.value.status == H.HJB_EINVAL
    with pytest.raises(H.HjbError) as e:
        H.hjb_solve_global(f, H.HJB_F32, v, opts=H.make_opts(patch_bc=H.HJB_BC_DIRICHLET))
    assert e.value.status == H.HJB_EINVAL
