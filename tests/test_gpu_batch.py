"""Batched form: the grouped launches of fcsph_batch_* give bitwise the
results of the plain per-plan calls, for a mix of sizes, wall types,
precisions, operator evaluations, 2D / 3D steps and PPE solves; the captured
HIP graph replays the next step bitwise like a second plain call."""
import numpy as np
import pytest

from gpu_helpers import lattice, rel_l2, spec, to_dev, to_np
from gpu_helpers import problem as _problem
from oracle import step
from paper_2606_06247_amd import synth

pytestmark = pytest.mark.gpu


def problem(s, **kw):
    """Every plan of these tests runs in batches (batched = 1)."""
    return _problem(s, batched=True, **kw)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2606_06247_amd import api
    assert torch.cuda.is_available()
    return api.Context(0)


def random_walls(rng):
    return tuple(tuple(rng.choice(["D", "N"]) for _ in range(2)) for _ in range(2))


def instances(seed=7):
    """(spec, precision, op_eval, kind) for a mixed batch; repeated shapes form
    groups; op_eval "fft+extended" is the whole-period route with the EXTENDED
    projection."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(14):
        n = int(rng.choice([64, 96, 128]))
        vel = random_walls(rng)
        prec = "fp64" if i % 3 else "fp32"
        oe = ["fft_window", "fft", "direct"][i % 3]
        out.append((spec((n, n), (True, True), vel=vel), prec, oe, "step"))
    for oe in ("fft_window", "fft_window", "fft"):
        out.append((spec((64, 64), (True, True), vel=(("D", "D"), ("D", "D"))), "fp64", oe, "step"))
    out.append((spec((24, 33, 16), (False, True, False), vel=(None, ("D", "N"), None)), "fp64", "fft_window", "step"))
    out.append((spec((32, 40, 24), (False, True, False)), "fp32", "fft", "step"))
    out.append((spec((96, 96), (True, True), vel=(("N", "D"), ("D", "D"))), "fp64", "fft_window", "ppe"))
    out.append((spec((96, 96), (True, True), vel=(("N", "D"), ("D", "D"))), "fp64", "fft_window", "ppe"))
    out.append((spec((64, 64), (True, True), vel=(("D", "N"), ("D", "D"))), "fp64", "fft+extended", "step"))
    out.append((spec((24, 33, 16), (False, True, False)), "fp64", "fft+extended", "step"))
    return out


def make_problem(s, prec, oe):
    if oe == "fft+extended":
        return problem(s, precision=prec, op_eval="fft", ppe_domain="extended")
    return problem(s, precision=prec, op_eval=oe)


def make_inputs(s, seed):
    if s["nd"] == 2:
        u = [synth.poly_trig_2d(s["n"], seed + k, dx=s["dx"]) for k in range(2)]
    else:
        u = list(synth.ChannelFlow3D(s["n"], seed, seed + 1).u)
    return u


def test_batch_matches_plain_calls_bitwise(ctx):
    import torch
    from paper_2606_06247_amd import api
    items = instances()
    plans = [api.Plan(ctx, make_problem(s, prec, oe)) for s, prec, oe, _ in items]
    dt, nu = 1e-4, 1e-3
    plain, batched, walls = [], [], []
    for i, (s, prec, oe, kind) in enumerate(items):
        u = make_inputs(s, 100 + 3 * i)
        if kind == "step":
            plain.append(([to_dev(c) for c in u], torch.zeros(tuple(reversed(s["n"])), dtype=torch.float64, device="cuda")))
            batched.append(([to_dev(c) for c in u], torch.zeros(tuple(reversed(s["n"])), dtype=torch.float64, device="cuda")))
            walls.append([to_dev(c) for c in u])
        else:
            rhs = to_dev(u[0])
            plain.append((rhs, None))
            batched.append((rhs, None))
            walls.append(None)
    # plain calls, one plan at a time
    plain_ppe = {}
    for i, (s, prec, oe, kind) in enumerate(items):
        if kind == "step":
            plans[i].project_step(plain[i][0], dt, nu, p_out=plain[i][1], wall=walls[i])
        else:
            plain_ppe[i] = plans[i].ppe_solve(plain[i][0])
    torch.cuda.synchronize()
    # one batch
    b = api.Batch(ctx, len(items))
    batch_ppe = {}
    for i, (s, prec, oe, kind) in enumerate(items):
        if kind == "step":
            b.add_step(plans[i], batched[i][0], dt, nu, p_out=batched[i][1], wall=walls[i])
        else:
            batch_ppe[i] = b.add_ppe(plans[i], batched[i][0])
    b.launch()
    torch.cuda.synchronize()
    n_items, n_groups, n_launch = b.info()
    assert n_items == len(items) and 1 < n_groups < len(items), (n_items, n_groups, n_launch)
    for i, (s, prec, oe, kind) in enumerate(items):
        if kind == "step":
            for a in range(s["nd"]):
                assert torch.equal(batched[i][0][a], plain[i][0][a]), (i, s["n"], prec, oe, a)
            assert torch.equal(batched[i][1], plain[i][1]), (i, "p")
        else:
            assert torch.equal(batch_ppe[i], plain_ppe[i]), (i, "ppe")
    # graph: the next step of every item by replay vs a second plain call
    b.capture()
    for i, (s, prec, oe, kind) in enumerate(items):
        if kind == "step":
            plans[i].project_step(plain[i][0], dt, nu, p_out=plain[i][1], wall=walls[i])
    torch.cuda.synchronize()
    b.replay()
    torch.cuda.synchronize()
    for i, (s, prec, oe, kind) in enumerate(items):
        if kind == "step":
            for a in range(s["nd"]):
                assert torch.equal(batched[i][0][a], plain[i][0][a]), ("replay", i, a)
    # replays with eager work in between: each replay advances the state once
    for rep in range(2):
        for i, (s, prec, oe, kind) in enumerate(items):
            if kind == "step":
                plans[i].project_step(plain[i][0], dt, nu, p_out=plain[i][1], wall=walls[i])
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        for i, (s, prec, oe, kind) in enumerate(items):
            if kind == "step":
                assert torch.equal(batched[i][1], plain[i][1]), ("replay p", rep, i)


def test_batch_step_against_oracle(ctx, fc_tables):
    """Two batched instances of different shapes and walls against the oracle."""
    import torch
    from paper_2606_06247_amd import api
    cases = [spec((64, 64), (True, True), vel=(("D", "N"), ("N", "D"))),
             spec((96, 96), (True, True), vel=(("N", "N"), ("D", "D")))]
    b = api.Batch(ctx, 4)
    plans, state, refs = [], [], []
    dt, nu = 1e-4, 1e-3
    for k, s in enumerate(cases):
        plan = api.Plan(ctx, problem(s, op_eval="fft_window"))
        u = make_inputs(s, 1000 + k)
        ud = [to_dev(c) for c in u]
        pd = torch.empty_like(ud[0])
        b.add_step(plan, ud, dt, nu, p_out=pd, wall=[to_dev(c) for c in u])
        plans.append(plan)
        state.append((ud, pd))
        refs.append(step.project_step(lattice(s), fc_tables, u, wall=u, dt=dt, nu=nu))
    b.launch()
    torch.cuda.synchronize()
    for (ud, pd), (ru, rp) in zip(state, refs):
        for a in range(2):
            assert rel_l2(to_np(ud[a]), ru[a]) < 1e-11
        assert rel_l2(to_np(pd), rp) < 1e-11


def test_batch_rejects_repeated_plan(ctx):
    import torch
    from paper_2606_06247_amd import api
    s = spec((64, 64), (True, True))
    plan = api.Plan(ctx, problem(s))
    b = api.Batch(ctx, 2)
    rhs = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    b.add_ppe(plan, rhs)
    with pytest.raises(api.FcsphError):
        b.add_ppe(plan, rhs)


def test_batch_tuned_schedules_bitwise(ctx):
    """Larger lattices, random walls, explicit window lengths, lines per
    workgroup and radix orders (the schedules the tuner picks; two items of
    one shape with different radix orders share a grouped launch):
    batched == plain bitwise."""
    import torch
    from paper_2606_06247_amd import api
    rng = np.random.default_rng(31)
    plans, plain, batched, walls = [], [], [], []
    for i, (n, L, lines, order) in enumerate([(192, 200, 1, 0), (192, 200, 1, 2), (256, 270, 2, 0),
                                              (384, 392, 1, 3), (256, 0, 0, 0)]):
        s = spec((n, n), (True, True), vel=random_walls(rng))
        prob = problem(s, op_eval="fft_window")
        prob.window_len = (L, L) if L else ()
        prob.lines_per_group = lines
        prob.radix_order = order
        plans.append(api.Plan(ctx, prob))
        u = make_inputs(s, 500 + 2 * i)
        plain.append([to_dev(c) for c in u])
        batched.append([to_dev(c) for c in u])
        walls.append([to_dev(c) for c in u])
    pp = [torch.empty_like(x[0]) for x in plain]
    pb = [torch.empty_like(x[0]) for x in plain]
    for i, plan in enumerate(plans):
        plan.project_step(plain[i], 1e-4, 1e-3, p_out=pp[i], wall=walls[i])
    b = api.Batch(ctx, len(plans))
    for i, plan in enumerate(plans):
        b.add_step(plan, batched[i], 1e-4, 1e-3, p_out=pb[i], wall=walls[i])
    b.launch()
    torch.cuda.synchronize()
    for i in range(len(plans)):
        for a in range(2):
            assert torch.equal(plain[i][a], batched[i][a]), (i, a, float((plain[i][a] - batched[i][a]).abs().max()))
        assert torch.equal(pp[i], pb[i]), i


@pytest.mark.parametrize("prec,oe", [("fp64", "fft_window"), ("fp32", "fft_window"), ("fp64", "fft")])
def test_tail_split_bitwise_1024(ctx, prec, oe):
    """At 1024^2 the one-problem stage-A column pass has more (field, column)
    tasks than resident workgroups on MI355X and splits the leftover tasks'
    outputs over separate workgroups; the grouped (batched) launch never
    splits.  Both must give the same step bitwise."""
    import torch
    from paper_2606_06247_amd import api
    s = spec((1024, 1024), (True, True), vel=(("D", "D"), ("D", "D")), prs=(("N", "N"), ("N", "N")))
    plan = api.Plan(ctx, problem(s, precision=prec, op_eval=oe))
    u = make_inputs(s, 77)
    plain = [to_dev(c) for c in u]
    batched = [to_dev(c) for c in u]
    wall = [to_dev(c) for c in u]
    pp, pb = torch.empty_like(plain[0]), torch.empty_like(plain[0])
    plan.project_step(plain, 1e-4, 1e-3, p_out=pp, wall=wall)
    b = api.Batch(ctx, 1)
    b.add_step(plan, batched, 1e-4, 1e-3, p_out=pb, wall=wall)
    b.launch()
    torch.cuda.synchronize()
    for a in range(2):
        assert torch.equal(plain[a], batched[a]), (a, float((plain[a] - batched[a]).abs().max()))
    assert torch.equal(pp, pb)


def test_batch_refuses_plan_with_streamed_ppe(ctx):
    """A plan built for single launches whose PPE uses the streamed radix
    stages (1023 = 31 x 11 x 3 at 1024^2) is refused by the batch calls, with
    no launch; built with batched = 1 it is accepted."""
    import torch
    from paper_2606_06247_amd import api
    s = spec((1024, 1024), (True, True), vel=(("D", "D"), ("D", "D")), prs=(("N", "N"), ("N", "N")))
    rhs = torch.zeros((1024, 1024), dtype=torch.float64, device="cuda")
    b = api.Batch(ctx, 2)
    single = api.Plan(ctx, _problem(s, op_eval="fft_window"))
    with pytest.raises(api.FcsphError, match="streamed"):
        b.add_ppe(single, rhs)
    b.add_ppe(api.Plan(ctx, problem(s, op_eval="fft_window")), rhs)
    b.launch()
    torch.cuda.synchronize()
