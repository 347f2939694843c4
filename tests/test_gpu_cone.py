"""Add-on AO3 (Section "Patchy method's add-ons"): each node minimises over
the controls in the cone of half-angle pi/r around its Step 2 feedback
control.  Parity of the HIP path with the oracle's solve_patches_cone: FP64
bit-exact (the cone membership is decided on the host in FP64 by the same
rule on both sides, and the FP64 kernel evaluates the candidates as the
oracle does), FP32 within 1e-5 of the FP64 oracle.
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
        return pr.variable_speed_2d(2, 193, 17, 32, 16, 0.1, True), 4.0
    if case == "2d_drift":
        return pr.variable_speed_2d(3, 150, 17, 20, 9, 0.1, True, drift_sign=1), 2.5
    if case == "2d_nc200":   # masks of four 64-bit words
        return pr.variable_speed_2d(4, 97, 17, 200, 6, 0.1, True), 6.0
    return pr.variable_speed_3d(0, 37, 11, 98, 4, 4, 0.25, True), 4.0


SHAPES = {"2d": [None, (32, 16, 1)], "2d_drift": [None, (32, 16, 1)], "2d_nc200": [None],
          "3d": [None]}


@pytest.mark.parametrize("case", ["2d", "2d_drift", "2d_nc200", "3d"])
def test_cone_solve_parity(H, orc, pr, case):
    (f, c), r = _case(pr, case)
    out = orc.patchy(f, c)
    ref, _ = orc.solve_patches_cone(f, out["labels"], out["feedback"], r)
    _, lmax = orc.cone_allowed(f, r)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    assert np.array_equal(ph.feedback(), out["feedback"])
    assert np.array_equal(ph.labels(), out["labels"])
    for tile in SHAPES[case]:
        print(f"[cone] {case} r={r} tile={tile}", flush=True)
        o = H.make_opts(tile=tile, threads=256 if tile else 0, control_cone=r)
        v64 = _zeros(f.N, True)
        st = H.hjb_solve_patches(f, ph, H.HJB_F64, v64, opts=o)
        assert np.array_equal(_np(v64), ref)
        assert st["updates"] == st["node_updates"] * lmax
        v32 = _zeros(f.N, False)
        H.hjb_solve_patches(f, ph, H.HJB_F32, v32, opts=o)
        assert np.abs(_np(v32) - ref).max() <= 1e-5
    # the cone only removes candidates: never below the basic result, and
    # the two differ somewhere (r is small enough to cut optimal controls)
    vb = _zeros(f.N, True)
    H.hjb_solve_patches(f, ph, H.HJB_F64, vb)
    assert np.all(_np(v64) >= _np(vb)) and np.any(_np(v64) != _np(vb))


def test_cone_line_target_exact(H, orc, pr):
    """Line target: the cone never removes the optimal control, so the AO3
    result is the basic one bit for bit (also in FP32: same candidates)."""
    f = pr.line_target_2d(97, 32, strips=3, fp32=True)
    c = pr.line_target_2d(25, 32, strips=3)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    for fp64 in (True, False):
        vb = _zeros(f.N, fp64)
        H.hjb_solve_patches(f, ph, H.HJB_F64 if fp64 else H.HJB_F32, vb)
        vc = _zeros(f.N, fp64)
        st = H.hjb_solve_patches(f, ph, H.HJB_F64 if fp64 else H.HJB_F32, vc,
                                 opts=H.make_opts(control_cone=4.5))
        assert np.array_equal(_np(vc), _np(vb))
        assert st["updates"] == st["node_updates"] * 7


def test_cone_r_at_most_one_is_basic(H, pr):
    f, c = pr.variable_speed_2d(1, 97, 17, 32, 8, 0.1, True)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    vb = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, vb)
    for r in (0.5, 1.0):
        v = _zeros(f.N, False)
        st = H.hjb_solve_patches(f, ph, H.HJB_F32, v, opts=H.make_opts(control_cone=r))
        assert np.array_equal(_np(v), _np(vb))
        assert st["updates"] == st["node_updates"] * 32


def test_cone_graph_and_patch_select(H, pr):
    """Graph replay of the rounds, and a subset of patches, give the same
    bits as the plain cone solve (patches are independent)."""
    f, c = pr.variable_speed_2d(5, 161, 17, 32, 8, 0.1, True)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    lab = ph.labels()
    v = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, v, opts=H.make_opts(control_cone=3.0))
    g = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, g, opts=H.make_opts(control_cone=3.0, use_graph=True))
    assert np.array_equal(_np(g), _np(v))
    sel = np.zeros(8, dtype=np.uint8)
    sel[[1, 6]] = 1
    s = _zeros(f.N, False)
    H.hjb_solve_patches(f, ph, H.HJB_F32, s,
                        opts=H.make_opts(control_cone=3.0, patch_select=sel))
    m = (lab == 1) | (lab == 6)
    assert np.array_equal(_np(s)[m], _np(v)[m])


def test_cone_rejections(H, pr):
    f, c = pr.variable_speed_2d(1, 65, 17, 16, 4, 0.1, True)
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    v = _zeros(f.N, False)
    bad = [H.make_opts(control_cone=4.0, schedule=H.HJB_SCHED_ASYNC),
           H.make_opts(control_cone=4.0, tile=(16, 16, 1), threads=256),
           H.make_opts(control_cone=-1.0),
           H.make_opts(control_cone=float("nan"))]
    for o in bad:
        with pytest.raises(H.HjbError) as e:
            H.hjb_solve_patches(f, ph, H.HJB_F32, v, opts=o)
        assert e.value.status == H.HJB_EINVAL
    with pytest.raises(H.HjbError) as e:
        H.hjb_solve_global(f, H.HJB_F32, v, opts=H.make_opts(control_cone=4.0))
    assert e.value.status == H.HJB_EINVAL
    with pytest.raises(H.HjbError) as e:
        H.hjb_batch_create([f], [c], opts=H.make_opts(control_cone=4.0))
    assert e.value.status == H.HJB_EINVAL
