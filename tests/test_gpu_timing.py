"""Kernel timing restricted to one kernel kind: the bench brackets only the
dominant kernel with events inside its timed region, so the restriction must
record that kind alone, once per launch."""
import pytest

from gpu_helpers import problem, spec

pytestmark = pytest.mark.gpu


def test_timing_only_one_kind():
    import torch
    from paper_2606_06247_amd import api
    ctx = api.Context(0)
    plan = api.Plan(ctx, problem(spec((64, 64), (True, True)), op_eval="fft_window"))
    g = torch.Generator(device="cpu").manual_seed(5)
    u = [torch.rand(64, 64, generator=g, dtype=torch.float64).cuda() for _ in range(2)]
    p = torch.empty_like(u[0])
    ctx.read_timing()
    ctx.set_timing(True)
    plan.project_step(u, 1e-4, 1e-3, p_out=p)
    ctx.set_timing(False)
    every = ctx.read_timing()
    assert "cols_op_step_a" in every and len(every) > 5, every
    ctx.set_timing(True, only="cols_op_step_a")
    plan.project_step(u, 1e-4, 1e-3, p_out=p)
    plan.project_step(u, 1e-4, 1e-3, p_out=p)
    ctx.set_timing(False)
    one = ctx.read_timing()
    assert set(one) == {"cols_op_step_a"} and one["cols_op_step_a"][0] == 2, one
    # set_timing(False) also cleared the restriction
    ctx.set_timing(True)
    plan.project_step(u, 1e-4, 1e-3, p_out=p)
    ctx.set_timing(False)
    assert set(ctx.read_timing()) == set(every)
    with pytest.raises(api.FcsphError):
        ctx.set_timing(True, only="x" * 40)
