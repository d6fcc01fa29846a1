"""Serving loop: every request served in a continuous-batching mix returns
bitwise the output of the same request run alone through the plain call, and
every request completes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_served_results_equal_alone(precision):
    import torch
    from paper_2606_06247_amd import api, serve
    reqs = serve.make_requests(lam=5000.0, count=40, seed=41, n2=(64, 160), n3=(32, 48))
    srv = serve.Server(precision, max_batch=8, lanes=2)
    srv.warm(sorted({(r.dims, r.n) for r in reqs}))
    stats = srv.run(reqs, realtime=True, keep_outputs=True)
    assert stats["requests"] == len(reqs)
    assert stats["batches"] >= 2
    assert all(np.isfinite(r.t_done) and r.t_done >= r.t_arrival for r in reqs)
    # alone: a fresh plan, the same inputs, the plain call
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
