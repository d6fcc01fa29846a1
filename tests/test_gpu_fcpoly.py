"""The paper's own FC (polynomial fit + quintic blend, d = 10 fit points,
degree 5, extension n / 4) through the C ABI against the oracle: the library
takes the package's maps (built by QR), the oracle its own (exact rational
normal equations)."""
import dataclasses

import numpy as np
import pytest

from gpu_helpers import check, fc_rounding_bound, gate, lattice, problem, rel_l2, spec, to_dev, to_np
from oracle import fc as ofc
from oracle import fcpoly, step
from paper_2606_06247_amd import synth

pytestmark = pytest.mark.gpu

D_FIT, DEG = 10, 5


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2606_06247_amd import api
    assert torch.cuda.is_available()
    return api.Context(0)


def setup(s, op_eval="fft_window", precision="fp64"):
    from paper_2606_06247_amd import api
    C = max(k for k, w in zip(s["n"], s["walled"]) if w) // 4
    prob = problem(s, precision=precision, op_eval=op_eval)
    prob.fc_kind, prob.fc_d, prob.fc_C, prob.fc_p = "poly", D_FIT, C, DEG
    lat = dataclasses.replace(lattice(s), C=C, d=D_FIT)
    return prob, lat, fcpoly.build(d=D_FIT, p=DEG, C=C)


CASES = [
    spec((64, 64), (True, True)),                                            # Dirichlet u, Neumann p
    spec((64, 64), (True, True), prs=(("D", "D"), ("D", "D"))),
    spec((72, 65), (True, True), vel=(("D", "N"), ("N", "D"))),              # quarter-wave pressure
    spec((48, 65), (False, True)),
]


@pytest.mark.parametrize("s", CASES[:3], ids=lambda s: f"{s['n']}-{s['vel']}")
def test_fc_extend_poly(ctx, s):
    from paper_2606_06247_amd import api
    prob, lat, tabs = setup(s)
    plan = api.Plan(ctx, prob)
    f = synth.poly_trig_2d(s["n"], 3, dx=s["dx"])
    for fc, bcs in ((api.VELOCITY, s["vel"]), (api.PRESSURE, s["prs"])):
        got = to_np(plan.fc_extend(to_dev(f), fc))
        ref = ofc.extend(f, s["walled"], bcs, tabs)
        assert got.shape == ref.shape
        ny, nx = f.shape
        assert np.array_equal(got[:ny, :nx], f)
        bound = fc_rounding_bound(f, lat, bcs, tabs)
        assert np.all(np.abs(got - ref) <= bound + 1e-300), float(np.max(np.abs(got - ref) - bound))


@pytest.mark.parametrize("op_eval", ["fft", "fft_window", "direct"])
@pytest.mark.parametrize("s", CASES, ids=lambda s: f"{s['n']}-{s['vel']}")
def test_project_step_poly(ctx, s, op_eval):
    import torch
    from paper_2606_06247_amd import api
    prob, lat, tabs = setup(s, op_eval)
    plan = api.Plan(ctx, prob)
    smooth = lambda seed: synth.poly_trig_2d(s["n"], seed, dx=s["dx"])  # noqa: E731
    u = [smooth(10), smooth(11)]
    f = [smooth(12), smooth(13)]
    w = [c.copy() for c in u]
    dt, nu = 1e-4, 1e-3
    ud = [to_dev(c) for c in u]
    pd = torch.empty_like(ud[0])
    plan.project_step(ud, dt, nu, p_out=pd, force=[to_dev(c) for c in f], wall=[to_dev(c) for c in w])
    ref_u, ref_p = step.project_step(lat, tabs, u, force=f, wall=w, dt=dt, nu=nu)
    fft_u, fft_p = (step.project_step(lat, tabs, u, force=f, wall=w, dt=dt, nu=nu, opmode="fft")
                    if op_eval == "fft" else ([None] * 2, None))
    for a in range(2):
        check(f"paper FC step u{a} {op_eval}", to_np(ud[a]), ref_u[a], gate(op_eval, ref_u[a], fft_u[a]))
    check(f"paper FC step p {op_eval}", to_np(pd), ref_p, gate(op_eval, ref_p, fft_p))


def _decaying_flow_1024_poly(ctx, op_eval):
    import torch
    from paper_2606_06247_amd import api
    n = 1024
    s = spec((n, n), (True, True))
    prob, lat, tabs = setup(s, op_eval)
    plan = api.Plan(ctx, prob)
    nu = 1e-3
    dx = 1.0 / (n - 1)
    dt = min(0.2 * dx, 0.1 * dx * dx / nu)
    flow = synth.DecayingVortexFlow(n, nu)
    u = list(flow.velocity(0.0))
    f = list(flow.force(0.5 * dt))
    w = list(flow.velocity(dt))
    ud = [to_dev(c) for c in u]
    pd = torch.empty_like(ud[0])
    plan.project_step(ud, dt, nu, p_out=pd, force=[to_dev(c) for c in f], wall=[to_dev(c) for c in w])
    ref_u, ref_p = step.project_step(lat, tabs, u, force=f, wall=w, dt=dt, nu=nu)
    for a in range(2):
        check(f"paper FC 1024^2 u{a} {op_eval}", to_np(ud[a]), ref_u[a], 1e-11)
    check(f"paper FC 1024^2 p {op_eval}", to_np(pd), ref_p, 1e-11)


def test_decaying_flow_1024_poly_window(ctx):
    """The 1024^2 workload with the paper's FC (extension 256 points) on the
    windowed route: the flat FP64 gate."""
    _decaying_flow_1024_poly(ctx, "fft_window")


@pytest.mark.xfail(run=False, reason="not at parity: the paper's FC extrapolates 256 points, its continuation of "
                   "the step's u* and phi reaches 5e7-2e8, and a DFT over the whole extended period rounds "
                   "relative to those values; measured 8.6e-4 / 5.2e-3 / 1.4e-3 against the oracle (whose own "
                   "FFT evaluation differs from its tap sums by 1e-2)")
def test_decaying_flow_1024_poly_whole_period(ctx):
    """The same step on the whole extended period 1280 = 2^8 5 (the paper's
    1.25 N)."""
    _decaying_flow_1024_poly(ctx, "fft")
