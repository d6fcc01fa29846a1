"""End-to-end validation of the Gaussian-kernel step against a closed-form
flow, through the GPU first-order projection step.

The paper's channel validations (Poiseuille, plane Couette) run the G4
kernel at h = 8 dx with walls; under the readings adopted here the step's
projection map then has spectral radius about 8 (``tests/
test_oracle_stability.py``), so those flows grow from rounding noise.  On a
lattice periodic on every axis the projection is stable, and the decaying
Taylor-Green vortex
    u = sin(k x) cos(k y) F,  v = -cos(k x) sin(k y) F,  F = exp(-2 nu k^2 t)
solves the incompressible Navier-Stokes equations exactly (its advection is
a gradient that the projection removes).  With the 4th-order consistent G4
kernel the step converges to it: the error against the closed form falls
as dt halves, toward the kernel's spatial floor (measured 2.1e-3, 6.1e-4,
4.3e-4 at dt = 0.01, 0.005, 0.0025 on 128^2), while the Wendland C2 kernel's
un-normalised lattice Laplacian (which does not annihilate constants at
h = 1.3 dx) decays the vortex away (relative error 1.0).  These are
validations against the mathematics, not parity with the oracle; the
measured errors are printed."""
import numpy as np
import pytest

from gpu_helpers import spec, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2606_06247_amd import api
    assert torch.cuda.is_available()
    return api.Context(0)


def taylor_green_error(ctx, n, kernel, nu, t_end, nsteps):
    import torch
    from paper_2606_06247_amd import api
    dx = 1.0 / n
    s = spec((n, n), (False, False), dx=dx, h=8.0 if kernel == "g4" else 1.3, kernel=kernel)
    plan = api.Plan(ctx, api.Problem(n=s["n"], walled=s["walled"], dx=dx, h_over_dx=s["h"], kernel=kernel,
                                     op_eval="fft"))
    k = 2 * np.pi
    x = (np.arange(n) * dx)[None, :]
    y = (np.arange(n) * dx)[:, None]
    u0 = np.sin(k * x) * np.cos(k * y)
    v0 = -np.cos(k * x) * np.sin(k * y)
    u = [to_dev(u0), to_dev(v0)]
    p = torch.empty_like(u[0])
    dt = t_end / nsteps
    for _ in range(nsteps):
        plan.project_step(u, dt, nu, p_out=p)
    F = np.exp(-2 * nu * k * k * t_end)
    err = np.sqrt(np.sum((to_np(u[0]) - u0 * F) ** 2 + (to_np(u[1]) - v0 * F) ** 2) /
                  np.sum((u0 * F) ** 2 + (v0 * F) ** 2))
    return float(err)


def test_taylor_green_decay_g4(ctx):
    n, nu, t_end = 128, 0.01, 0.5
    e1 = taylor_green_error(ctx, n, "g4", nu, t_end, 50)
    e2 = taylor_green_error(ctx, n, "g4", nu, t_end, 100)
    e4 = taylor_green_error(ctx, n, "g4", nu, t_end, 200)
    wend = taylor_green_error(ctx, n, "wendland_c2", nu, t_end, 200)
    print(f"Taylor-Green at t = {t_end} (nu = {nu}, {n}^2): relative L2 error G4 dt = 0.01 / 0.005 / 0.0025: "
          f"{e1:.3e} / {e2:.3e} / {e4:.3e}; Wendland C2 at dt = 0.0025: {wend:.3e}")
    # the error falls with dt toward the spatial floor of G4 at h = 8 dx on
    # 128^2 (its gradient symbol is 1 - 7e-4 at this wavenumber)
    assert e4 < e2 < e1
    assert e4 < 1e-3
    assert e4 < 0.01 * wend
