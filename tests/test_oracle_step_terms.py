"""Pins of the terms of the intermediate velocity u* (no GPU).

Sec. "Temporal discretisation", eqs. uStarRK3 and rhsMomtem (first-order
coefficients a = g = 1, z = 0, sign reading of eq. IncompressibleNS):
    u* = u - dt [ (u . grad) u - nu lap u - f ].

On an all-periodic lattice (no FC) a velocity whose components are a constant
and a single Fourier mode along another axis is divergence-free under the SPH
divergence (a constant has zero SPH gradient: the gradient taps are odd; a
function of x alone has zero SPH y-derivative for the same reason), so the PPE
right-hand side vanishes, phi = 0 and u^{n+1} = u*.  The terms of u* then have
closed forms in three scalars of the operators on that mode, each measured by
applying the (separately pinned) oracle operators to the mode:
    G_x sin(theta x) = -beta cos(theta x),   L sin(theta x) = lam sin(theta x),
    L 1 = s0.
For u = (c, A sin(theta x)) and forcing f = (fx, B sin(theta x)):
    (u . grad) u = (0, -c A beta cos(theta x)),   lap u = (c s0, A lam sin(theta x)),
    u*_x = c + dt (nu c s0 + fx),
    u*_y = A sin(theta x) + dt (c A beta cos(theta x) + nu A lam sin(theta x) + B sin(theta x)).
A flipped viscous or forcing sign, or the transposed advection sum_b u_b G_a u_b
(which gives a nonzero x term A^2 beta sin cos), each changes the result at
O(dt).  The low-storage RK3 sub-step is pinned the same way through the F it
returns and through u after sub-step 0, u* = u - dt (g_0 F - a_0 f).
"""
import numpy as np
import pytest

from oracle import operators, step
from oracle.lattice import Lattice


def _case(ndim, mode_axis, along_axis):
    """All-periodic lattice; mode sin(theta x_m) along lattice axis `mode_axis`
    in velocity component `along_axis` (!= mode_axis)."""
    n = (18, 20) if ndim == 2 else (14, 16, 12)
    lat = Lattice(n=n, walled=(False,) * ndim, dx=1.0 / 16)
    m = 3
    idx = np.indices(lat.shape)                       # numpy order (.., y, x)
    xm = idx[ndim - 1 - mode_axis]
    theta = 2 * np.pi * m / n[mode_axis]
    return lat, np.sin(theta * xm), np.cos(theta * xm)


def _scalars(lat, sinm, cosm, mode_axis):
    ops = operators.Operators(lat, None)
    g = ops.grad(sinm)
    beta = -float(np.sum(g[mode_axis] * cosm) / np.sum(cosm * cosm))
    assert np.max(np.abs(g[mode_axis] + beta * cosm)) < 1e-12 * abs(beta)
    for a in range(lat.ndim):
        if a != mode_axis:
            assert np.max(np.abs(g[a])) < 1e-12 * abs(beta)
    lapm = ops.lap(sinm)
    lam = float(np.sum(lapm * sinm) / np.sum(sinm * sinm))
    assert np.max(np.abs(lapm - lam * sinm)) < 1e-12 * abs(lam)
    s0 = float(ops.lap(np.ones(lat.shape))[(0,) * lat.ndim])
    assert abs(beta) > 1.0 and abs(lam) > 1.0 and abs(s0) > 1.0    # every term is visible
    return beta, lam, s0


CASES = [(2, 0, 1), (2, 1, 0), (3, 0, 1), (3, 2, 0), (3, 1, 2)]


@pytest.mark.parametrize("ndim,mode_axis,comp", CASES)
def test_project_step_ustar_terms(ndim, mode_axis, comp):
    lat, sinm, cosm = _case(ndim, mode_axis, comp)
    beta, lam, s0 = _scalars(lat, sinm, cosm, mode_axis)
    A, B, nu, dt = 0.8, 2.5, 0.03, 0.01
    consts = [0.7, -0.4, 0.3]
    fconst = [0.9, -1.3, 0.6]
    u, f, exp = [], [], []
    c = consts[mode_axis]        # the velocity component along the mode axis is the constant c
    for a in range(ndim):
        if a == comp:
            u.append(A * sinm)
            f.append(B * sinm)
            # (u . grad) u_comp = c G_mode(A sin) = -c A beta cos
            exp.append(A * sinm + dt * (c * A * beta * cosm + nu * A * lam * sinm + B * sinm))
        else:
            ca = consts[a]
            u.append(np.full(lat.shape, ca))
            f.append(np.full(lat.shape, fconst[a]))
            exp.append(np.full(lat.shape, ca + dt * (nu * ca * s0 + fconst[a])))
    unew, phi = step.project_step(lat, None, u, force=f, dt=dt, nu=nu, family="sph")
    assert np.max(np.abs(phi)) < 1e-9
    scale = max(np.max(np.abs(e)) for e in exp)
    for a in range(ndim):
        assert np.max(np.abs(unew[a] - exp[a])) < 1e-12 * scale, a


@pytest.mark.parametrize("ndim,mode_axis,comp", CASES[:3])
def test_rk3_substep_terms(ndim, mode_axis, comp):
    lat, sinm, cosm = _case(ndim, mode_axis, comp)
    beta, lam, s0 = _scalars(lat, sinm, cosm, mode_axis)
    A, B, nu, dt = 0.8, 2.5, 0.03, 0.01
    consts = [0.7, -0.4, 0.3]
    c = consts[mode_axis]
    u, f, Fexp, uexp = [], [], [], []
    a0, g0 = step.RK3_A[0], step.RK3_G[0]
    for a in range(ndim):
        if a == comp:
            u.append(A * sinm)
            f.append(B * sinm)
            F = -c * A * beta * cosm - nu * A * lam * sinm
        else:
            u.append(np.full(lat.shape, consts[a]))
            f.append(np.full(lat.shape, 0.5))
            F = np.full(lat.shape, -nu * consts[a] * s0)
        Fexp.append(F)
        uexp.append(u[a] - dt * (g0 * F - a0 * f[a]))
    unew, phi, Fgot = step.rk3_substep(lat, None, u, 0, force=f, dt=dt, nu=nu, family="sph")
    for a in range(ndim):
        sF = np.max(np.abs(Fexp[a]))
        assert np.max(np.abs(Fgot[a] - Fexp[a])) < 1e-12 * sF, a
        assert np.max(np.abs(unew[a] - uexp[a])) < 1e-12 * np.max(np.abs(uexp[a])), a


def test_first_order_step_is_forward_euler_on_forced_shear_mode():
    """A forced shear mode u = (y0 cos(theta y), 0), f = (B cos(theta y), 0)
    is an eigenmode of every operator and has no advection: one step gives
    y1 = (1 + nu lam dt) y0 + dt B exactly."""
    lat = Lattice(n=(16, 20), walled=(False, False), dx=1.0 / 20)
    y = np.indices(lat.shape)[0]
    mode = np.cos(2 * np.pi * 3 * y / 20)
    lam = float(np.sum(operators.Operators(lat, None).lap(mode) * mode) / np.sum(mode * mode))
    y0, B, nu, dt = 1.3, -2.0, 0.05, 0.02
    unew, _ = step.project_step(lat, None, [y0 * mode, 0 * mode], force=[B * mode, 0 * mode],
                                dt=dt, nu=nu, family="sph")
    y1 = (1 + nu * lam * dt) * y0 + dt * B
    assert abs(nu * lam * dt) > 1e-3
    assert np.max(np.abs(unew[0] - y1 * mode)) < 1e-13 * abs(y1)
    assert np.max(np.abs(unew[1])) < 1e-13 * abs(y1)
