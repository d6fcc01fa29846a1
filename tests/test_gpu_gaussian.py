"""The Gaussian kernel family (G4..G10, h = 8 dx, infinite support sampled at
the minimum image over the whole extended lattice) through the C ABI
against the oracle, on the whole-period route: operators and steps with
FC(Gram) and with the paper's own FC, and the paper's operator convergence
test on eq. testFun10 run on the GPU.

Gate: the whole-period one (1e-11, or 20x the oracle's own FFT-vs-tap-sum
difference on the input when that is larger)."""
import dataclasses
import math

import numpy as np
import pytest

from gpu_helpers import check, gate, lattice, problem, spec, to_dev, to_np
from oracle import fcpoly, operators, step
from paper_2606_06247_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2606_06247_amd import api
    assert torch.cuda.is_available()
    return api.Context(0)


def with_fc(s, fc):
    """(library Problem, oracle Lattice, oracle FC tables) for FC(Gram) or the
    paper's FC (10 fit points, degree 5, extension n / 4 of the walled axis)."""
    prob = problem(s, op_eval="fft")
    lat = lattice(s)
    if fc == "gram":
        from oracle import fcgram
        return prob, lat, fcgram.load()
    C = max(k for k, w in zip(s["n"], s["walled"]) if w) // 4
    prob.fc_kind, prob.fc_d, prob.fc_C, prob.fc_p = "poly", 10, C, 5
    return prob, dataclasses.replace(lat, C=C, d=10), fcpoly.build(d=10, p=5, C=C)


OP_CASES = [
    (spec((40, 33), (True, True), vel=(("D", "N"), ("N", "D")), h=8.0, kernel="g4"), "gram"),
    (spec((64, 64), (True, True), h=8.0, kernel="g8"), "gram"),
    (spec((48, 37), (False, True), h=8.0, kernel="g6"), "gram"),
    (spec((24, 20), (False, False), dx=0.05, h=3.0, kernel="g10"), "gram"),
    (spec((64, 65), (False, True), dx=1.0 / 64, h=8.0, kernel="g4"), "poly"),
    (spec((72, 65), (True, True), vel=(("D", "N"), ("N", "D")), h=8.0, kernel="g4"), "poly"),
]


@pytest.mark.parametrize("s,fc", OP_CASES, ids=[f"{s['n']}-{s['kernel']}-{fc}" for s, fc in OP_CASES])
def test_gaussian_operators(ctx, s, fc):
    from paper_2606_06247_amd import api
    prob, lat, tabs = with_fc(s, fc)
    plan = api.Plan(ctx, prob)
    ops = operators.Operators(lat, tabs)
    opf = operators.Operators(lat, tabs, mode="fft")
    if all(s["walled"]) and s["n"][0] == s["n"][1]:
        f, g = synth.poly_trig_2d(s["n"], 2, dx=s["dx"]), synth.poly_trig_2d(s["n"], 3, dx=s["dx"])
    else:
        f, g = synth.poly_trig_2d(s["n"], 2, dx=s["dx"]), synth.poly_trig_2d(s["n"], 3, dx=s["dx"])
    tag = f"{s['kernel']} {s['n']} {fc}"
    for fc_class, name in ((api.VELOCITY, "u"), (api.PRESSURE, "p")):
        got = [to_np(t) for t in plan.spectral_grad(to_dev(f), fc_class)]
        ref, reff = ops.grad(f, name), opf.grad(f, name)
        for a in range(2):
            check(f"{tag} grad{a} {name}", got[a], ref[a], gate("fft", ref[a], reff[a]))
        lap = to_np(plan.spectral_lap(to_dev(f), fc_class))
        check(f"{tag} lap {name}", lap, ops.lap(f, name), gate("fft", ops.lap(f, name), opf.lap(f, name)))
    div = to_np(plan.spectral_div([to_dev(f), to_dev(g)]))
    check(f"{tag} div", div, ops.div([f, g]), gate("fft", ops.div([f, g]), opf.div([f, g])))


STEP_CASES = [
    (spec((64, 64), (True, True), h=8.0, kernel="g4"), "gram"),
    (spec((64, 65), (False, True), dx=1.0 / 64, h=8.0, kernel="g4"), "poly"),
    (spec((48, 37), (False, True), h=8.0, kernel="g8"), "gram"),
]


@pytest.mark.parametrize("s,fc", STEP_CASES, ids=[f"{s['n']}-{s['kernel']}-{fc}" for s, fc in STEP_CASES])
def test_gaussian_step(ctx, s, fc):
    import torch
    from paper_2606_06247_amd import api
    prob, lat, tabs = with_fc(s, fc)
    plan = api.Plan(ctx, prob)
    u = [synth.poly_trig_2d(s["n"], 10 + k, dx=s["dx"]) for k in range(2)]
    f = [synth.poly_trig_2d(s["n"], 12 + k, dx=s["dx"]) for k in range(2)]
    w = [c.copy() for c in u]
    dt, nu = 1e-4, 1e-3
    ud = [to_dev(c) for c in u]
    pd = torch.empty_like(ud[0])
    plan.project_step(ud, dt, nu, p_out=pd, force=[to_dev(c) for c in f], wall=[to_dev(c) for c in w])
    ref_u, ref_p = step.project_step(lat, tabs, u, force=f, wall=w, dt=dt, nu=nu)
    fu, fp = step.project_step(lat, tabs, u, force=f, wall=w, dt=dt, nu=nu, opmode="fft")
    tag = f"{s['kernel']} {s['n']} {fc}"
    for a in range(2):
        check(f"{tag} step u{a}", to_np(ud[a]), ref_u[a], gate("fft", ref_u[a], fu[a]))
    check(f"{tag} step p", to_np(pd), ref_p, gate("fft", ref_p, fp))


def _testfun10(n):
    nx, ny = n - 1, n
    dx = 1.0 / (n - 1)
    x = (np.arange(nx) * dx)[None, :]
    y = (np.arange(ny) * dx)[:, None]
    a, da, dda = y * (1 - y), 1 - 2 * y, -2.0 + 0 * y
    b = y ** 2 * (1 - y) ** 2
    db = 2 * y * (1 - y) ** 2 - 2 * y ** 2 * (1 - y)
    ddb = 2 * (1 - y) ** 2 - 8 * y * (1 - y) + 2 * y ** 2
    s2, c2 = np.sin(2 * np.pi * x), np.cos(2 * np.pi * x)
    c4, s4 = np.cos(4 * np.pi * x), np.sin(4 * np.pi * x)
    f = s2 * a + 0.5 * c4 * b
    fx = 2 * np.pi * c2 * a - 2 * np.pi * s4 * b
    fy = s2 * da + 0.5 * c4 * db
    lap = -(2 * np.pi) ** 2 * s2 * a + s2 * dda - 0.5 * (4 * np.pi) ** 2 * c4 * b + 0.5 * c4 * ddb
    return (nx, ny), dx, f, (fx, fy, lap)


def test_testfun10_convergence_on_gpu(ctx):
    """The paper's operator convergence test on the GPU (G4, h = 8 dx, the
    paper's FC with extension n/4): away from the walls (middle 40 % of y)
    the gradient and Laplacian errors fall at 4th order; the 257-point
    lattice also matches the oracle."""
    from paper_2606_06247_amd import api
    errs = {}
    for n in (257, 513, 1025):
        shape, dx, f, ref = _testfun10(n)
        s = spec(shape, (False, True), dx=dx, h=8.0, kernel="g4")
        prob, lat, tabs = with_fc(s, "poly")
        plan = api.Plan(ctx, prob)
        fd = to_dev(f)
        g = [to_np(t) for t in plan.spectral_grad(fd)]
        lp = to_np(plan.spectral_lap(fd))
        band = slice(int(0.3 * shape[1]), int(0.7 * shape[1]))
        rms = lambda e: float(np.sqrt(np.mean(e[band] ** 2)))   # noqa: E731
        errs[n] = (rms(g[0] - ref[0]), rms(g[1] - ref[1]), rms(lp - ref[2]))
        if n == 257:
            opf = operators.Operators(lat, tabs, mode="fft")
            og = opf.grad(f)
            for a in range(2):
                check(f"testFun10 G4 257 grad{a} vs oracle", g[a], og[a], 1e-11)
            check("testFun10 G4 257 lap vs oracle", lp, opf.lap(f), 1e-11)
    print("testFun10 G4 interior RMS errors (grad x, grad y, lap):", errs)
    for a, b in ((257, 513), (513, 1025)):
        orders = [math.log2(ea / eb) for ea, eb in zip(errs[a], errs[b])]
        print(f"  orders {a}->{b}:", [f"{o:.2f}" for o in orders])
        assert all(3.5 < o < 4.6 for o in orders), (a, b, orders)
