"""Pins of the oracle's linear advection (no GPU).

P-ADV1: on a lattice periodic on every axis a Fourier mode e^{i theta . j} is
        an eigenvector of the SPH gradient, G_a e = S_a e (S_a measured by
        applying the pinned operator to the mode), so one RK3 step maps it to
        R(z) e with z = -dt (c . S) and R(z) = 1 + z + z^2/2 + z^3/6 (any
        three-stage third-order scheme on y' = lambda y).  A wrong sign of the
        advection term, a wrong g_k or z_k, or a dropped F recursion changes
        R at O(z).
P-ADV2: inflow walls carry the imposed data after every sub-step, outflow
        walls do not.

A finding, not a pin: the linear map of one RK3 step on the walled unit
square (inflow data zero, CFL 0.5) has spectral radius below one with the
Wendland C2 kernel at h = 1.3 dx and about 63 with the Gaussian G4 kernel at
h = 2 dx, the same at 13 and 25 points a side (a wall mode: the G4 stencil
reaches the continuation values far from the wall, whose FC(Gram) rows carry
entries up to 3.4e3 times the boundary data).
"""
import numpy as np
import pytest

from oracle import advect, operators
from oracle.lattice import Lattice, walled_box


@pytest.mark.parametrize("c", [(1.0, 0.5), (-0.7, 0.3), (0.4, -1.1)])
def test_rk3_amplification_of_a_fourier_mode(c):
    n = (18, 20)
    lat = Lattice(n=n, walled=(False, False), dx=1.0 / 18)
    j = np.indices(lat.shape)                     # numpy order (y, x)
    th = (2 * np.pi * 3 / n[0], 2 * np.pi * 2 / n[1])
    phase = th[0] * j[1] + th[1] * j[0]
    cosm, sinm = np.cos(phase), np.sin(phase)
    ops = operators.Operators(lat, None)
    gc, gs = ops.grad(cosm), ops.grad(sinm)
    e = np.exp(1j * phase)
    S = [complex(np.mean((gc[a] + 1j * gs[a]) / e)) for a in range(2)]
    for a in range(2):
        assert np.max(np.abs(gc[a] + 1j * gs[a] - S[a] * e)) < 1e-12 * abs(S[a])
    dt = 1.0 / abs(c[0] * S[0] + c[1] * S[1])      # |z| = 1: every term of R matters
    z = -dt * (c[0] * S[0] + c[1] * S[1])
    R = 1 + z + z * z / 2 + z ** 3 / 6
    # evolve the real and imaginary parts (the scheme is real-linear)
    out = []
    for u0 in (cosm, sinm):
        u, F = u0.copy(), None
        for k in range(3):
            u, F = advect.rk3_substep(lat, None, u, k, c, F_prev=F, dt=dt)
        out.append(u)
    got = out[0] + 1j * out[1]
    assert np.max(np.abs(got - R * e)) < 1e-12 * np.max(np.abs(R * e))
    assert abs(R - np.exp(z)) > 1e-3               # the cubic differs from the exponential here


def test_inflow_walls_take_the_data(fc_tables):
    n = 21
    lat = walled_box((n, n))
    rng = np.random.default_rng(4)
    u = rng.standard_normal((n, n))
    wall = rng.standard_normal((n, n))
    c = (1.0, -0.5)                                  # inflow: x = 0 (low x) and y = 1 (high y)
    F = None
    for k in range(3):
        u, F = advect.rk3_substep(lat, fc_tables, u, k, c, F_prev=F, wall=wall, dt=1e-3)
        assert np.array_equal(u[:, 0], wall[:, 0])
        assert np.array_equal(u[-1, :], wall[-1, :])
        assert not np.array_equal(u[1:-1, -1], wall[1:-1, -1])      # outflow x = 1
        assert not np.array_equal(u[0, 1:-1], wall[0, 1:-1])        # outflow y = 0


def _step_map(lat, tables, c, dt):
    N = lat.shape[0] * lat.shape[1]
    A = np.zeros((N, N))
    for i in range(N):
        u = np.zeros(N)
        u[i] = 1.0
        u, F = u.reshape(lat.shape), None
        for k in range(3):
            u, F = advect.rk3_substep(lat, tables, u, k, c, F_prev=F, wall=None, dt=dt, opmode="fft")
        A[:, i] = u.ravel()
    return A


@pytest.mark.parametrize("kernel,h,lo,hi", [("wendland_c2", 1.3, 0.99, 1.0), ("g4", 2.0, 63.1, 63.2)])
def test_step_map_radius(fc_tables, kernel, h, lo, hi):
    lat = walled_box((13, 13), h_over_dx=h, kernel=kernel)
    A = _step_map(lat, fc_tables, (1.0, 0.5), 0.5 * lat.dx)
    r = np.max(np.abs(np.linalg.eigvals(A)))
    print(kernel, h, "spectral radius", r)
    assert lo < r < hi
