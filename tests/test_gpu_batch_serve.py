"""Batched solves and the continuous-batching server through the C ABI.

Both pack work items of many problems into shared sweep rounds.  Every
update is monotone and items write only their own patch of their own
problem, so each result must equal, bit for bit, the same problem solved
alone -- whatever else is in the mix, and whenever it joins."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available()
    from paper_1109_3577_amd import hjb
    return hjb


def _alone(H, f, c, precision):
    import torch
    ch = H.hjb_coarse_solve(c)
    ph = H.hjb_build_patches(f, ch)
    v = torch.empty(f.N, dtype=torch.float32 if precision == H.HJB_F32 else torch.float64,
                    device="cuda")
    H.hjb_solve_patches(f, ph, precision, v)
    return v.cpu().numpy(), ph.labels()


def _mixed_problems(pr, k=6):
    """Uneven 2D problems (sizes, controls, parts, drift) plus 3D ones."""
    ss = np.random.SeedSequence(11).spawn(k)
    probs = [pr.batched_problem(s, i, (65, 200)) for i, s in enumerate(ss)]
    probs.append(pr.variable_speed_3d(3, 29, 9, 98, 2, 4, 0.3, True, "b3d"))
    probs.append(pr.variable_speed_2d(9, 97, 17, 32, 16, 0.1, True))
    return probs


def test_batch_equals_alone_fp32(H, pr):
    probs = _mixed_problems(pr)
    b = H.hjb_batch_create([f for f, _ in probs], [c for _, c in probs], H.HJB_F32)
    st = H.hjb_batch_run(b)
    assert st["status"] == H.HJB_OK and st["updates"] > 0
    for i, (f, c) in enumerate(probs):
        got, sti = H.hjb_batch_result(b, i)
        ref, _ = _alone(H, f, c, H.HJB_F32)
        assert np.array_equal(got, ref), i
        assert sti["updates"] > 0


def test_batch_equals_oracle_fp64(H, orc, pr):
    probs = _mixed_problems(pr, 3)[:3]
    b = H.hjb_batch_create([f for f, _ in probs], [c for _, c in probs], H.HJB_F64)
    H.hjb_batch_run(b)
    for i, (f, c) in enumerate(probs):
        got, _ = H.hjb_batch_result(b, i)
        assert np.array_equal(got, orc.patchy(f, c)["v"]), i


def test_server_same_alone_and_in_mix(H, pr):
    """Requests arrive while others are live; each finishes with the bits
    of its solve alone, and the HBM budget bounds what is admitted."""
    probs = _mixed_problems(pr, 5)
    S = H.hjb_server_create(2 << 30, H.HJB_F32)
    tickets = {}
    done = {}
    pending = list(enumerate(probs))
    steps = 0
    while pending or len(done) < len(probs):
        if pending:  # one new request per step, while earlier ones run
            i, (f, c) = pending.pop(0)
            tickets[i] = S.submit(f, c)
        live, queued = S.step(2)
        steps += 1
        for i, t in list(tickets.items()):
            if i in done:
                continue
            v, st = S.poll(t)
            if v is not None:
                done[i] = (v, st)
        assert steps < 10000
    for i, (f, c) in enumerate(probs):
        ref, _ = _alone(H, f, c, H.HJB_F32)
        assert np.array_equal(done[i][0], ref), i
        assert done[i][1]["status"] == H.HJB_OK


def test_server_admission_by_budget(H, pr):
    """A request larger than the whole budget is refused up front; with a
    budget for one request at a time, requests run one after the other."""
    f, c = pr.variable_speed_2d(0, 129, 17, 16, 4, 0.1, True)
    S = H.hjb_server_create(1 << 20, H.HJB_F32)
    with pytest.raises(H.HjbError) as e:
        S.submit(f, c)
    assert e.value.status == H.HJB_EINVAL
    # one 129^2 request holds about 2.7 MB (values, inputs, labels and the
    # transient colour/feedback buffers of its build step)
    S = H.hjb_server_create(4 << 20, H.HJB_F32)
    t1 = S.submit(f, c)
    t2 = S.submit(f, c)
    # the first request is prepared in the background, then joins the live
    # rounds; the second waits for budget the whole time
    for _ in range(5000):
        live, queued = S.step(1)
        assert live + queued == 2 or live == 1
        if live:
            break
    assert live == 1 and queued == 1
    out = {}
    for _ in range(2000):
        for t in (t1, t2):
            if t not in out:
                v, _ = S.poll(t)
                if v is not None:
                    out[t] = v
        if len(out) == 2:
            break
        S.step(4)
    assert np.array_equal(out[t1], out[t2])


@pytest.mark.parametrize("prepare_bytes", [1, 10 << 20])
def test_batch_preparation_chunks_equal_alone(H, pr, prepare_bytes):
    """The shared colour transport of a batch's preparation in chunks (one
    problem per chunk, or a few): every result keeps the bits of its solve
    alone."""
    probs = _mixed_problems(pr)
    b = H.hjb_batch_create([f for f, _ in probs], [c for _, c in probs], H.HJB_F32,
                           prepare_bytes=prepare_bytes)
    H.hjb_batch_run(b)
    for i, (f, c) in enumerate(probs):
        got, _ = H.hjb_batch_result(b, i)
        ref, _ = _alone(H, f, c, H.HJB_F32)
        assert np.array_equal(got, ref), i


@pytest.mark.parametrize("sched", ["graph", "async"])
def test_batch_schedules_bitwise(H, pr, sched):
    """The batch in other launch forms: its rounds captured once and replayed
    as a hipGraph (solve.use_graph), and all of its items drained by one
    persistent launch per dimension (HJB_SCHED_ASYNC).  Every schedule of the
    monotone iteration stops at the same fixed point, so each problem's
    values equal the plain rounds' bit for bit: FP32 and FP64, 2D and 3D
    problems, state constraint and the Dirichlet data of eq. dbc."""
    import torch
    probs = _mixed_problems(pr, 4)
    fs, cs = [f for f, _ in probs], [c for _, c in probs]
    s = torch.cuda.Stream()
    for prec in (H.HJB_F32, H.HJB_F64):
        for bc in (H.HJB_BC_STATE, H.HJB_BC_DIRICHLET):
            ref = H.hjb_batch_create(fs, cs, prec, 0.0, 0, H.make_opts(patch_bc=bc), stream=s)
            H.hjb_batch_run(ref)
            kw = {"use_graph": True} if sched == "graph" else {"schedule": H.HJB_SCHED_ASYNC}
            b = H.hjb_batch_create(fs, cs, prec, 0.0, 0, H.make_opts(patch_bc=bc, **kw), stream=s)
            st = H.hjb_batch_run(b)
            assert st["status"] == H.HJB_OK
            for i in range(len(probs)):
                want, _ = H.hjb_batch_result(ref, i)
                got, _ = H.hjb_batch_result(b, i)
                assert np.array_equal(got, want), (prec, bc, i)
            b.free()
            ref.free()


def test_server_refuses_async(H):
    with pytest.raises(H.HjbError):
        H.hjb_server_create(1 << 30, H.HJB_F32, 0.0, 0, H.make_opts(schedule=H.HJB_SCHED_ASYNC))


def test_server_failed_request_leaves_others(H, pr):
    """A request whose data fail the per-node checks (a non-finite speed,
    found by the preparation pool) is collected with its error; its budget
    is released, and the requests around it finish with the bits of their
    solves alone."""
    import copy
    f, c = pr.variable_speed_2d(1, 129, 17, 16, 4, 0.1, True)
    bad = copy.deepcopy(f)
    bad.speed = np.array(bad.speed, dtype=np.float64)
    bad.speed[777] = np.nan
    S = H.hjb_server_create(6 << 20, H.HJB_F32)
    t1 = S.submit(f, c)
    tb = S.submit(bad, c)
    t2 = S.submit(f, c)
    out, err = {}, {}
    for _ in range(5000):
        S.step(4)
        for t in (t1, tb, t2):
            if t in out or t in err:
                continue
            try:
                v, st = S.poll(t)
            except H.HjbError as e:
                err[t] = e
                continue
            if v is not None:
                out[t] = v
        if len(out) + len(err) == 3:
            break
    assert set(err) == {tb} and err[tb].status == H.HJB_EINVAL
    ref, _ = _alone(H, f, c, H.HJB_F32)
    assert np.array_equal(out[t1], ref) and np.array_equal(out[t2], ref)
