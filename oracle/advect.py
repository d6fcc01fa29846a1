"""Linear advection with inflow / outflow walls (oracle side).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

Sec. "Gaussian vortex convection", eqs. linearAdvection and
GaussianVortexAnalytical: a scalar u is transported with the constant
velocity (C_x, C_y) across the non-periodic unit square,
    du/dt + C_x du/dx + C_y du/dy = 0,
from the Gaussian u_0 = exp(-alpha r^2), r^2 = (x - x_0)^2 + (y - y_0)^2,
whose exact solution is u_0 translated by (C_x t, C_y t).  Readings of the
garbled formulas: the second advection term is C_y du/dy (printed with d/dx),
the initial Gaussian decays (exp(-alpha r^2), printed exp(alpha r^2)), and
the exponent of the exact solution covers both squared offsets (the printed
bracket closes after the first).  The method: the field is FC-extended
(FC(Gram) or the paper's own FC) and differentiated by the spectral SPH
gradient (``oracle.operators``), and advanced by the low-storage RK3 of the
temporal discretisation section:
    F^k = C . grad u^k,   u^{k+1} = u^k - dt (g_k F^k + z_k F^{k-1}),
Readings of the boundary treatment (the section states none): the
transported scalar carries no wall condition of its own, so every wall uses
the plain continuation map (M_D: values only, no derivative condition); the
inflow walls (where C . n < 0, n the outward normal) take the exact solution
at the end of each sub-step; the outflow walls keep the computed values.

Parity: pinned in ``tests/test_oracle_advect.py`` by the RK3 stability
polynomial on a periodic Fourier mode (amplification R(-dt C . S) with S the
gradient symbols: fixes the sign of the advection term, the RK3 weights and
the F recursion) and by the wall rule (inflow walls hold the imposed data
after every sub-step, outflow walls do not).  The gradient itself is the
pinned operator of ``oracle.operators``.
"""
from __future__ import annotations

import numpy as np

from . import operators
from .step import RK3_G, RK3_Z


def inflow_walls(lat, c):
    """Per walled axis (low, high): True where the wall is an inflow wall."""
    out = []
    for a in range(lat.ndim):
        if not lat.walled[a]:
            out.append((False, False))
        else:
            out.append((c[a] > 0, c[a] < 0))
    return tuple(out)


def set_walls(f, lat, mask, wall):
    f = f.copy()
    nd = lat.ndim
    for a in range(nd):
        ax = nd - 1 - a
        for side, on in zip((0, -1), mask[a]):
            if on:
                sl = [slice(None)] * nd
                sl[ax] = side
                f[tuple(sl)] = 0.0 if wall is None else wall[tuple(sl)]
    return f


def rk3_substep(lat, tables, u, k, c, F_prev=None, wall=None, dt=1e-3, opmode: str = "direct"):
    """Sub-step k (0, 1, 2) of the RK3 step of length dt (u: the scalar, c:
    the velocity per lattice axis, wall: the exact solution at the end of the
    sub-step for the inflow walls).  Returns (u_new, F)."""
    import dataclasses
    # every wall continued with the plain (value) map
    lat_d = dataclasses.replace(lat, vel_bc=tuple(("D", "D") if w else None for w in lat.walled))
    ops = operators.Operators(lat_d, tables, mode=opmode)
    g = ops.grad(np.asarray(u, dtype=np.float64), "u")
    F = sum(c[a] * g[a] for a in range(lat.ndim))
    Fp = 0.0 if (k == 0 or F_prev is None) else F_prev
    unew = u - dt * (RK3_G[k] * F + RK3_Z[k] * Fp)
    return set_walls(unew, lat, inflow_walls(lat, c), wall), F

