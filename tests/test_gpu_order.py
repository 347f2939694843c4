"""Value-ordered schedule (add-on AO2, Section "Patchy method's add-ons"):
tiles run in the order of their Step 2 values.  Only the order of the
monotone updates changes, so the result is the same fixed point: FP64 bit
for bit the oracle's, FP32 bit for bit the unordered FP32 result.
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
    if case == "2d":
        return pr.variable_speed_2d(2, 193, 17, 32, 16, 0.1, True)
    if case == "2d_drift":
        return pr.variable_speed_2d(3, 150, 17, 20, 9, 0.1, True, drift_sign=1)
    return pr.variable_speed_3d(0, 37, 11, 98, 4, 4, 0.25, True)


@pytest.mark.parametrize("case", ["2d", "2d_drift", "3d"])
def test_ordered_same_fixed_point(H, orc, pr, case):
    f, c = _case(pr, case)
    out = orc.patchy(f, c)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    v32 = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, v32)
    for w in (1.0, 5.0, 1e9):
        print(f"[order] {case} window {w}", flush=True)
        o = H.make_opts(order_window=w)
        v64 = _zeros(f.N, True)
        st = H.hjb_solve_patches(f, ph, H.HJB_F64, v64, opts=o)
        assert st["status"] == H.HJB_OK
        assert np.array_equal(_np(v64), out["v"])
        w32 = _zeros(f.N, False)
        H.hjb_solve_patches(f, ph, H.HJB_F32, w32, opts=o)
        assert np.array_equal(_np(w32), _np(v32))


def test_ordered_with_cone_dbc_graph(H, orc, pr):
    f, c = pr.variable_speed_2d(6, 161, 17, 32, 8, 0.1, True)
    out = orc.patchy(f, c)
    ref, _ = orc.solve_patches_ex(f, out["labels"], out["feedback"], 4.0, out["u0"])
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    for graph in (False, True):
        o = H.make_opts(order_window=3.0, control_cone=4.0, patch_bc=H.HJB_BC_DIRICHLET,
                        use_graph=graph)
        v64 = _zeros(f.N, True)
        H.hjb_solve_patches(f, ph, H.HJB_F64, v64, opts=o)
        assert np.array_equal(_np(v64), ref)


def test_ordered_tolerance_stop(H, orc, pr):
    """With tol > 0 the ordered run stops above the fixed point, within the
    bound of the stopping rule."""
    f, c = pr.variable_speed_2d(1, 129, 17, 32, 8, 0.1, True)
    out = orc.patchy(f, c)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    v64 = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, v64, 1e-6, opts=H.make_opts(order_window=3.0))
    d = _np(v64) - out["v"]
    assert d.min() >= 0.0 and d.max() <= 1e-6 / (1.0 - f.beta)


def test_ordered_rejections(H, pr):
    f, c = pr.variable_speed_2d(1, 65, 17, 16, 4, 0.1, True)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    v = _zeros(f.N, False)
    for o in (H.make_opts(order_window=0.1, schedule=H.HJB_SCHED_ASYNC),
              H.make_opts(order_window=-1.0), H.make_opts(order_window=float("inf"))):
        with pytest.raises(H.HjbError) as e:
            H.hjb_solve_patches(f, ph, H.HJB_F32, v, opts=o)
        assert e.value.status == H.HJB_EINVAL
    with pytest.raises(H.HjbError) as e:
        H.hjb_solve_global(f, H.HJB_F32, v, opts=H.make_opts(order_window=0.1))
    assert e.value.status == H.HJB_EINVAL


def test_ordered_batch_and_server_equal_alone(H, pr):
    """The ordered schedule in a batch and in the server: every problem
    keeps the FP32 bits of its unordered solve alone."""
    probs = [pr.variable_speed_2d(7, 97, 17, 24, 6, 0.1, True),
             pr.variable_speed_2d(8, 130, 17, 32, 12, 0.1, True, drift_sign=-1),
             pr.variable_speed_3d(3, 29, 9, 98, 2, 4, 0.3, True, "b3d")]
    alone = []
    for f, c in probs:
        ch = H.hjb_coarse_solve(c)
        ph = H.hjb_build_patches(f, ch)
        v = _zeros(f.N, False)
        H.hjb_solve_patches(f, ph, H.HJB_F32, v)
        alone.append(v.cpu().numpy())
    o = H.make_opts(order_window=3.0)
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
