"""Pins of the oracle's low-storage RK3 sub-steps (no GPU).

P-RK1 : on an all-periodic lattice a shear mode u = (A cos(2 pi m y / L), 0)
        with forcing (B cos(2 pi m y / L), 0) is an eigenmode of every operator
        of the step (no advection, no divergence), so the step reduces to the
        scalar affine ODE y' = mu y + B with mu = nu lambda (lambda: the SPH
        Laplacian's eigenvalue of the mode).  Any three-stage third-order
        Runge-Kutta scheme maps it exactly to
            y_3 + B / mu = R(mu dt) (y_0 + B / mu),  R(x) = 1 + x + x^2/2 + x^3/6.
        A wrong coefficient, a dropped z_k F^{k-1} term or a wrong forcing
        weight changes R or the forced part at O(1).
P-RK2 : all-periodic lattice with the SPH eigenvalue family: after every
        sub-step the new velocity is SPH-divergence-free to rounding, which
        holds only if the a_k of the PPE and of the correction cancel.
"""
import numpy as np

from oracle import operators, step
from oracle.lattice import Lattice


def _shear_case():
    nx, ny, m = 16, 20, 3
    lat = Lattice(n=(nx, ny), walled=(False, False), dx=1.0 / ny)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    mode = np.cos(2 * np.pi * m * y / ny)
    return lat, mode


def test_rk3_stability_polynomial_on_forced_shear_mode():
    lat, mode = _shear_case()
    ops = operators.Operators(lat, None)
    lap = ops.lap(mode)
    lam = float(np.sum(lap * mode) / np.sum(mode * mode))
    assert np.max(np.abs(lap - lam * mode)) < 1e-12 * abs(lam)       # an eigenmode
    nu, dt, A, B = 1e-2, 0.15, 0.7, 3.0
    mu = nu * lam
    x = mu * dt
    assert -1.2 < x < -0.4                                           # the cubic term matters
    u = [A * mode, np.zeros_like(mode)]
    f = [B * mode, np.zeros_like(mode)]
    F = None
    for k in range(3):
        u, phi, F = step.rk3_substep(lat, None, u, k, F_prev=F, force=f, dt=dt, nu=nu, family="sph")
    R = 1 + x + x * x / 2 + x ** 3 / 6
    y3 = R * (A + B / mu) - B / mu
    amp = float(np.sum(u[0] * mode) / np.sum(mode * mode))
    assert abs(amp - y3) < 1e-12 * max(abs(y3), 1.0), (amp, y3)
    assert np.max(np.abs(u[0] - amp * mode)) < 1e-12 * abs(amp)
    assert np.max(np.abs(u[1])) < 1e-12 * abs(amp)
    # the exponential differs from the cubic by x^4 / 24: the pin separates them
    assert abs(np.exp(x) * (A + B / mu) - B / mu - y3) > 1e-4


def test_rk3_projection_divergence_free_every_substep():
    lat = Lattice(n=(20, 16), walled=(False, False), dx=1.0 / 20)
    ops = operators.Operators(lat, None)
    rng = np.random.default_rng(5)
    u = [rng.standard_normal((16, 20)) for _ in range(2)]
    scale = np.max(np.abs(ops.div(u)))
    F = None
    for k in range(3):
        u, phi, F = step.rk3_substep(lat, None, u, k, F_prev=F, dt=1e-3, nu=1e-2, family="sph")
        assert np.max(np.abs(ops.div(u))) < 1e-11 * scale, k
        assert np.max(np.abs(phi)) > 0


def test_rk3_dirichlet_walls(fc_tables):
    from oracle.lattice import walled_box
    from paper_2606_06247_amd import synth
    n = 17
    lat = walled_box((n, n), vel_bc=(("D", "D"), ("N", "D")))
    u = [synth.poly_trig_2d(n, seed=s) for s in (1, 2)]
    w = [synth.poly_trig_2d(n, seed=s) for s in (3, 4)]
    F = None
    for k in range(3):
        u, phi, F = step.rk3_substep(lat, fc_tables, u, k, F_prev=F, wall=w, dt=1e-4, nu=1e-3)
        for c in range(2):
            assert np.array_equal(u[c][:, 0], w[c][:, 0]) and np.array_equal(u[c][:, -1], w[c][:, -1])
            assert np.array_equal(u[c][-1, :], w[c][-1, :])
            assert not np.array_equal(u[c][0, 1:-1], w[c][0, 1:-1])   # y low wall is Neumann
