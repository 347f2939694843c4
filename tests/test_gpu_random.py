"""Seeded random instances through the whole path, against the oracle:
grid sizes that leave ragged tiles, 4-64 controls, 1-40 target parts of
every size, drift in either sense, 2D and 3D.  Labels and the Step 2
values are compared bit for bit, the merged values of Steps 3.2-4 bit for
bit in FP64 and within 1e-5 in FP32, the eq. dbc solve and the control
cones of add-on AO3 (r = 4) bit for bit in FP64, and the value-ordered
schedule of add-on AO2 bit for bit against the plain one."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(20261203)
    out = []
    for i in range(32):
        if i % 4 == 3:
            n = int(rng.integers(17, 41))
            out.append(("3d", dict(seed=int(rng.integers(0, 1000)), n=n,
                                   nc_coarse=int(rng.integers(5, 10)),
                                   nc=int(rng.choice([14, 26, 50, 98])),
                                   bands=int(rng.integers(1, 4)), sectors=int(rng.integers(1, 5)),
                                   r=float(rng.uniform(0.2, 0.4)))))
        else:
            n = int(rng.integers(20, 151))
            out.append(("2d", dict(seed=int(rng.integers(0, 1000)), n=n,
                                   nc_coarse=int(rng.integers(9, 34)),
                                   nc=int(rng.integers(4, 65)), R=int(rng.integers(1, 41)),
                                   r=float(rng.uniform(0.05, 0.3)),
                                   drift=[None, 1, -1][int(rng.integers(0, 3))])))
    return out


CASES = _cases()


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available()
    from paper_1109_3577_amd import hjb
    return hjb


@pytest.mark.parametrize("i", range(len(CASES)))
def test_random_instance(H, orc, pr, i):
    import torch
    kind, p = CASES[i]
    print(f"[random] case {i}: {kind} {p}", flush=True)
    if kind == "2d":
        f, c = pr.variable_speed_2d(p["seed"], p["n"], p["nc_coarse"], p["nc"], p["R"], p["r"],
                                    True, p["drift"])
    else:
        f, c = pr.variable_speed_3d(p["seed"], p["n"], p["nc_coarse"], p["nc"], p["bands"],
                                    p["sectors"], p["r"], True)
    out = orc.patchy(f, c)
    ch = H.hjb_coarse_solve(c)
    assert np.array_equal(ch.values(), out["v_coarse"])
    ph = H.hjb_build_patches(f, ch)
    assert np.array_equal(ph.u0(), out["u0"])
    assert np.array_equal(ph.labels(), out["labels"])
    v64 = torch.empty(f.N, dtype=torch.float64, device="cuda")
    H.hjb_solve_patches(f, ph, H.HJB_F64, v64)
    assert np.array_equal(v64.cpu().numpy(), out["v"])
    v32 = torch.empty(f.N, dtype=torch.float32, device="cuda")
    H.hjb_solve_patches(f, ph, H.HJB_F32, v32)
    assert np.abs(v32.double().cpu().numpy() - out["v"]).max() <= 1e-5
    ref, _ = orc.solve_patches_ex(f, out["labels"], u0=out["u0"])
    d64 = torch.empty(f.N, dtype=torch.float64, device="cuda")
    H.hjb_solve_patches(f, ph, H.HJB_F64, d64, opts=H.make_opts(patch_bc=H.HJB_BC_DIRICHLET))
    assert np.array_equal(d64.cpu().numpy(), ref)
    cone, _ = orc.solve_patches_cone(f, out["labels"], out["feedback"], 4.0)
    c64 = torch.empty(f.N, dtype=torch.float64, device="cuda")
    H.hjb_solve_patches(f, ph, H.HJB_F64, c64, opts=H.make_opts(control_cone=4.0))
    assert np.array_equal(c64.cpu().numpy(), cone)
    o64 = torch.empty(f.N, dtype=torch.float64, device="cuda")
    H.hjb_solve_patches(f, ph, H.HJB_F64, o64, opts=H.make_opts(order_window=6.0))
    assert np.array_equal(o64.cpu().numpy(), out["v"])
