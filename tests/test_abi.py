"""The C-ABI library: it loads, exports every declared symbol, and rejects
malformed arguments with HJB_EINVAL before touching the GPU (CPU tests)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hjb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hjb_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def H():
    from paper_1109_3577_amd import hjb
    return hjb


def test_library_exports_every_declared_symbol(H):
    decl = _declared()
    assert len(decl) >= 20
    for name in decl:
        assert hasattr(H.lib, name), name
    assert set(decl) == set(H.EXPORTS)
    assert "gfx950" in H.hjb_version()


def test_struct_layouts_match_header(H, tmp_path):
    """Every field offset and struct size of the binding equals what a C
    compiler gives the structs of include/hjb.h."""
    import subprocess
    structs = {"hjb_problem": H.hjb_problem, "hjb_stats": H.hjb_stats,
               "hjb_solve_opts": H.hjb_solve_opts, "hjb_batch_opts": H.hjb_batch_opts,
               "hjb_server_opts": H.hjb_server_opts, "hjb_build_opts": H.hjb_build_opts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hjb.h"', "int main(void){"]
    for sname, cls in structs.items():
        lines.append(f'printf("{sname} sizeof %zu\\n", sizeof({sname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{sname} {f} %zu\\n", offsetof({sname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = {}
    for line in out.splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for sname, cls in structs.items():
        assert got[(sname, "sizeof")] == C.sizeof(cls), sname
        for f, _ in cls._fields_:
            assert got[(sname, f)] == getattr(cls, f).offset, (sname, f)


def _bad_problem(pr, **kw):
    P = pr.eikonal_2d(17, 8, 0.3)
    for k, v in kw.items():
        setattr(P, k, v)
    return P


@pytest.mark.parametrize("field,value,msg", [
    ("dim", 4, "dim"),
    ("beta", 1.5, "beta"),
    ("omb", 0.123, "one_minus_beta"),
    ("n_parts", 0, "n_parts"),
])
def test_invalid_descriptor_rejected(H, pr, field, value, msg):
    P = _bad_problem(pr)
    hp = H.Problem(P)
    if field == "omb":
        hp.s.one_minus_beta = value
    elif field == "dim":
        hp.s.dim = value
    else:
        setattr(hp.s, field, value)
    with pytest.raises(H.HjbError) as e:
        H.hjb_coarse_solve(hp)
    assert e.value.status == H.HJB_EINVAL
    assert msg in str(e.value)


def test_reach_beyond_halo_rejected(H, pr):
    P = pr.eikonal_2d(17, 8, 0.3)
    P.speed = np.full(P.N, 2.5)
    with pytest.raises(H.HjbError) as e:
        H.hjb_coarse_solve(P)
    assert e.value.status == H.HJB_EINVAL and "reach" in str(e.value)


def test_nonfinite_and_bad_parts_rejected(H, pr):
    P = pr.eikonal_2d(17, 8, 0.3)
    P.speed = P.speed.copy()
    P.speed[5] = np.nan
    with pytest.raises(H.HjbError):
        H.hjb_coarse_solve(P)
    P = pr.eikonal_2d(17, 8, 0.3, R=2)
    tp = P.target_part.copy()
    tp[tp >= 0] = 5
    P.target_part = tp
    with pytest.raises(H.HjbError) as e:
        H.hjb_coarse_solve(P)
    assert "n_parts" in str(e.value)


def test_too_many_controls_rejected(H, pr):
    P = pr.eikonal_2d(17, 300, 0.3)
    with pytest.raises(H.HjbError) as e:
        H.hjb_coarse_solve(P)
    assert "n_controls" in str(e.value)


def test_null_output_rejected(H):
    assert H.lib.hjb_coarse_solve(None, 0.0, 0, None, None) == H.HJB_EINVAL
    assert "NULL" in H.last_error()
    assert H.lib.hjb_patches_labels(None, None, 0) == H.HJB_EINVAL
    assert H.lib.hjb_server_poll(None, 1, None, 0, None) == H.HJB_EINVAL


def test_constants_match_header(H):
    """Every #define HJB_* integer constant of include/hjb.h that the
    binding names has the same value there."""
    src = open(os.path.join(ROOT, "include", "hjb.h")).read()
    defs = dict(re.findall(r"#define\s+(HJB_[A-Z0-9_]+)\s+(-?\d+)\b", src))
    names = [n for n in defs if hasattr(H, n)]
    assert {"HJB_BC_STATE", "HJB_BC_DIRICHLET", "HJB_SCHED_ASYNC", "HJB_F64"} <= set(names)
    for n in names:
        assert getattr(H, n) == int(defs[n]), n
