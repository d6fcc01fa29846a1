"""Serving loop: every request served in a continuous-batching mix returns
bitwise the output of the same request run alone through the plain call, and
every request completes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def assert_equal_alone(srv, reqs, precision):
    """Every served output equals bitwise the plain call on a fresh plan with
    the same inputs."""
    import torch
    from paper_2606_06247_amd import api, serve
    ctx = api.Context(0)
    for r in reqs:
        plan = api.Plan(ctx, serve.problem_for(r.dims, r.n, precision))
        bufs = srv._inputs(r)
        if r.kind == "step":
            plan.project_step(bufs["u"], srv.dt, srv.nu, p_out=bufs["p"], wall=bufs["wall"])
            ref = bufs["u"] + [bufs["p"]]
        else:
            ref = [plan.ppe_solve(bufs["rhs"], bufs["phi"])]
        torch.cuda.synchronize()
        got = r.out[0] + [r.out[1]] if r.kind == "step" else r.out
        assert len(got) == len(ref)
        for g, f in zip(got, ref):
            assert torch.equal(g, f), (r.rid, r.kind, r.dims, r.n)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_served_results_equal_alone(precision):
    from paper_2606_06247_amd import serve
    reqs = serve.make_requests(lam=5000.0, count=40, seed=41, n2=(64, 160), n3=(32, 48))
    srv = serve.Server(precision, max_batch=8, lanes=2)
    srv.warm(sorted({(r.dims, r.n) for r in reqs}))
    stats = srv.run(reqs, realtime=True, keep_outputs=True)
    assert stats["requests"] == len(reqs)
    assert stats["batches"] >= 2
    assert all(np.isfinite(r.t_done) and r.t_done >= r.t_arrival for r in reqs)
    assert_equal_alone(srv, reqs, precision)


def test_lone_requests_take_the_plain_call():
    """Requests that arrive one at a time run alone on their plan's lane as
    the plain call (no grouped batch), with the same results."""
    from paper_2606_06247_amd import serve
    reqs = serve.make_requests(lam=100.0, count=6, seed=43, n2=(64, 96), n3=(32, 40))
    srv = serve.Server("fp64", max_batch=8, lanes=2)
    srv.warm(sorted({(r.dims, r.n) for r in reqs}))
    stats = srv.run(reqs, realtime=True, keep_outputs=True)
    assert stats["status"].get("ok", 0) == len(reqs)
    assert srv.stats.get("plain_launches", 0) >= 1
    assert_equal_alone(srv, reqs, "fp64")


def test_admission_respects_budget():
    """With a budget that holds one plan of each shape plus little else, the
    server still completes every request (requests wait for idle plans)."""
    import torch
    from paper_2606_06247_amd import api, serve
    reqs = serve.make_requests(lam=5000.0, count=16, seed=42, p_2d=1.0, n2=(64, 96))
    shapes = sorted({(r.dims, r.n) for r in reqs})
    # room for the resident plans and the buffers of one request (less than
    # the smallest plan workspace): no second plan of any shape fits
    req_bytes = max(r.n ** 2 * 8 * 5 for r in reqs)
    lanes = 2
    budget = lanes * sum(api.workspace_bytes(serve.problem_for(d, n, "fp64")) for d, n in shapes) + req_bytes
    srv = serve.Server("fp64", hbm_budget=budget, max_batch=8, lanes=lanes)
    srv.warm(shapes)
    stats = srv.run(reqs, realtime=False)
    assert stats["requests"] == len(reqs)
    assert stats["plans_created"] == lanes * len(shapes)
    assert srv.used <= budget


def test_nonfinite_request_fails_alone():
    """A request whose input carries a NaN ends "nonfinite" (the library's
    finiteness count on its outputs); every other request of the same
    batches ends "ok" with the output it has alone."""
    import torch
    from paper_2606_06247_amd import api, serve
    reqs = serve.make_requests(lam=5000.0, count=24, seed=43, p_2d=1.0, n2=(64, 96))
    for r in reqs[3::7]:
        r.poison = True
    srv = serve.Server("fp64", max_batch=8, lanes=2, check_finite=True)
    srv.warm(sorted({(r.dims, r.n) for r in reqs}))
    stats = srv.run(reqs, realtime=False, keep_outputs=True)
    print("status counts", stats["status"])
    assert stats["status"].get("nonfinite", 0) == len(reqs[3::7])
    assert stats["status"].get("ok", 0) == len(reqs) - len(reqs[3::7])
    ctx = api.Context(0)
    for r in reqs:
        assert r.status == ("nonfinite" if r.poison else "ok"), (r.rid, r.status)
        if r.poison:
            continue
        plan = api.Plan(ctx, serve.problem_for(r.dims, r.n, "fp64"))
        bufs = srv._inputs(r)
        if r.kind == "step":
            plan.project_step(bufs["u"], srv.dt, srv.nu, p_out=bufs["p"], wall=bufs["wall"])
            ref = bufs["u"] + [bufs["p"]]
            got = r.out[0] + [r.out[1]]
        else:
            ref = [plan.ppe_solve(bufs["rhs"], bufs["phi"])]
            got = r.out
        torch.cuda.synchronize()
        for g, f in zip(got, ref):
            assert torch.equal(g, f), r.rid


def test_check_finite_counts():
    import torch
    from paper_2606_06247_amd import api, serve
    plan = api.Plan(api.Context(0), serve.problem_for(2, 64, "fp64"))
    x = torch.zeros(100003, dtype=torch.float64, device="cuda")
    assert plan.nonfinite_count(x) == 0
    x[[0, 17, 50000, 100002]] = torch.tensor([float("nan"), float("inf"), float("-inf"), float("nan")],
                                            dtype=torch.float64, device="cuda")
    assert plan.nonfinite_count(x) == 4


def test_rejection_timeout_and_cancel():
    """Requests that can never fit the budget are refused on arrival; queued
    requests past their admission deadline time out; cancelled queued
    requests leave; everything else completes."""
    from paper_2606_06247_amd import api, serve
    reqs = serve.make_requests(lam=5000.0, count=30, seed=44, p_2d=1.0, n2=(64, 80))
    shapes = sorted({(r.dims, r.n) for r in reqs})
    lanes = 1
    budget = lanes * sum(api.workspace_bytes(serve.problem_for(d, n, "fp64")) for d, n in shapes) + 1e6
    big = serve.Request(1000, 0.0, "step", 2, 512, 7)          # its plan alone exceeds the room left
    reqs.append(big)
    for r in reqs[:20]:
        r.t_arrival = 0.0
    reqs[5].deadline = 0.0                                    # cannot be admitted in time
    srv = serve.Server("fp64", hbm_budget=budget, max_batch=2, lanes=lanes)
    srv.warm(shapes)
    srv.cancel(reqs[12].rid)
    stats = srv.run(reqs, realtime=True)
    print("status counts", stats["status"])
    assert big.status == "rejected"
    assert reqs[12].status == "cancelled"
    assert reqs[5].status in ("timeout", "ok")
    assert stats["status"].get("ok", 0) >= len(reqs) - 3
    assert all(r.status != "pending" for r in reqs)
    assert srv.used <= budget
