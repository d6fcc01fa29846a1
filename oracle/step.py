"""One first-order projection (FOP) step (oracle side).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

Sec. "Temporal discretisation": eqs. uStarRK3, rhsMomtem, PPE and u^n+1 with
the first-order projection coefficients a = g = 1, z = 0 stated after the RK3
table.  Readings of the garbled signs and terms:
* u* = u - dt [ (u . grad) u - nu lap u - f ]  (signs consistent with eq.
  IncompressibleNS; the pressure term of eq. uStarRK3 is dropped because FOP is
  the non-incremental Chorin projection, so phi is the new pressure);
* lap phi = (rho / dt) div u*;  u^{n+1} = u* - (dt / rho) grad phi;
* Dirichlet velocity wall points of u* and of u^{n+1} are set to the wall data
  at t^{n+1}; Neumann velocity walls are left as computed.

Spatial operators: spectral SPH gradient / Laplacian on FC-extended fields
(``oracle.operators``), velocity FC for u and u*, pressure FC for phi.

Modes:
* 'physical' (the paper's solver): phi from the PPE on the physical lattice
  (``oracle.ppe``), then extended by pressure FC to take its gradient;
* 'extended' (the fully periodic alternative the paper mentions at the end of
  Sec. "Integration of Fourier continuation ..."): the projection is done on the
  extended periodic lattice in Fourier space with the SPH symbols,
  phi_hat = (rho/dt) D / sum_a S_a^2 with D = sum_a S_a u*_hat_a (modes whose
  symbol sum vanishes are left untouched), u_hat -= (dt/rho) S_a phi_hat.  This
  definition is spectral, so the oracle uses numpy's FFT for it.

Low-storage RK3 (``rk3_substep``): the same equations with the RK3
coefficient table of that section, sub-step k = 0, 1, 2:
* F^k = (u^k . grad) u^k - nu lap u^k  (sign reading as above);
* u* = u^k - dt [ g_k F^k + z_k F^{k-1} - a_k f ]  (pressure term dropped as
  in the first-order form; f is the forcing averaged over the sub-step);
* lap phi = rho / (a_k dt) div u*  (a_k read as dividing dt, the form that
  makes u^{k+1} below divergence-free; identical for a_k = 1);
* u^{k+1} = u* - a_k (dt / rho) grad phi;  Dirichlet walls as above.

Parity: built from pinned parts (operators, PPE, FC); the step itself is pinned
by the projection identities P-PRJ1/P-PRJ2 and by direct-vs-fft mode agreement
in ``tests/test_oracle_step.py``, and its u* terms (advection order, viscous
and forcing signs, in 2D and 3D) by closed forms on single Fourier modes of an
all-periodic lattice in ``tests/test_oracle_step_terms.py``.  The RK3 sub-steps are pinned by the
stability polynomial 1 + z + z^2/2 + z^3/6 of a three-stage third-order
scheme on a forced linear shear mode, and by the projected velocity being
divergence-free to rounding on an all-periodic lattice with the SPH
eigenvalue family (``tests/test_oracle_rk3.py``); the F it returns and the
first sub-step's u* by the same single-mode closed forms as the first-order
step.  Multi-step trajectories:
parity unpinned beyond those.
"""
from __future__ import annotations

import numpy as np

from . import fc as fcmod
from . import operators, ppe


def set_dirichlet_walls(f: np.ndarray, lat, wall: np.ndarray | None) -> np.ndarray:
    """Copy wall data into the Dirichlet velocity wall points of f."""
    f = f.copy()
    nd = lat.ndim
    for a in range(nd):
        if not lat.walled[a]:
            continue
        ax = nd - 1 - a
        for side, bc in zip((0, -1), lat.vel_bc[a]):
            if bc != "D":
                continue
            sl = [slice(None)] * nd
            sl[ax] = side
            sl = tuple(sl)
            f[sl] = 0.0 if wall is None else wall[sl]
    return f


def project_step(lat, tables, u, force=None, wall=None, dt=1e-4, nu=1e-3, rho=1.0,
                 mode: str = "physical", family: str = "spectral", opmode: str = "direct",
                 return_parts: bool = False):
    """One FOP step.  u: list of velocity components (numpy arrays, physical
    shape); force, wall: lists of the same shape or None.  Returns (u_new, p)."""
    ops = operators.Operators(lat, tables, mode=opmode)
    nd = lat.ndim
    u = [np.asarray(c, dtype=np.float64) for c in u]
    grads = [ops.grad(c, "u") for c in u]            # grads[a][b] = G_b u_a
    laps = [ops.lap(c, "u") for c in u]
    ustar = []
    for a in range(nd):
        adv = sum(u[b] * grads[a][b] for b in range(nd))
        F = adv - nu * laps[a]
        fa = 0.0 if force is None else force[a]
        us = u[a] - dt * (F - fa)
        ustar.append(set_dirichlet_walls(us, lat, None if wall is None else wall[a]))
    parts = dict(ustar=ustar, grads=grads, laps=laps)
    if mode == "physical":
        b = (rho / dt) * ops.div(ustar)
        phi, diag = ppe.solve(b, lat, family=family, return_diag=True)
        gphi = ops.grad(phi, "p")
        unew = []
        for a in range(nd):
            un = ustar[a] - (dt / rho) * gphi[a]
            unew.append(set_dirichlet_walls(un, lat, None if wall is None else wall[a]))
        parts.update(b=b, phi=phi, gphi=gphi, bhat0=diag["bhat0"])
        return (unew, phi, parts) if return_parts else (unew, phi)
    if mode == "extended":
        ext_shape = lat.ext_shape
        S = []
        for a in range(nd):
            ker = operators.corner_wrapped_kernel(ext_shape, ops.grad_taps[a])
            S.append(np.fft.fftn(ker))
        ehat = [np.fft.fftn(ops.extend(c, "u")) for c in ustar]
        D = sum(S[a] * ehat[a] for a in range(nd))
        ssq = sum(S[a] * S[a] for a in range(nd)).real
        tol = 1e-14 * np.max(np.abs(ssq))
        ok = np.abs(ssq) > tol
        phihat = np.where(ok, (rho / dt) * D / np.where(ok, ssq, 1.0), 0.0)
        unew = []
        uhat_new = []
        for a in range(nd):
            uh = ehat[a] - (dt / rho) * S[a] * phihat
            uhat_new.append(uh)
            un = fcmod.restrict(np.fft.ifftn(uh).real, lat.n)
            unew.append(set_dirichlet_walls(un, lat, None if wall is None else wall[a]))
        phi = fcmod.restrict(np.fft.ifftn(phihat).real, lat.n)
        parts.update(S=S, uhat_new=uhat_new, D=D, phihat=phihat)
        return (unew, phi, parts) if return_parts else (unew, phi)
    raise ValueError(mode)


# RK3 coefficient table of the temporal discretisation section
RK3_A = (8.0 / 15.0, 2.0 / 15.0, 1.0 / 3.0)
RK3_G = (8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0)
RK3_Z = (0.0, -17.0 / 60.0, -5.0 / 12.0)


def rk3_substep(lat, tables, u, k, F_prev=None, force=None, wall=None, dt=1e-4, nu=1e-3, rho=1.0,
                family: str = "spectral", opmode: str = "direct", return_parts: bool = False):
    """Sub-step k (0, 1, 2) of the low-storage RK3 step of length dt.
    u: velocity components; F_prev: F of the previous sub-step (ignored for
    k = 0); force: forcing averaged over the sub-step; wall: Dirichlet data at
    the end of the sub-step.  Returns (u_new, phi, F), plus a dict with u*
    and the PPE right-hand side b when return_parts is set."""
    a, g, z = RK3_A[k], RK3_G[k], RK3_Z[k]
    ops = operators.Operators(lat, tables, mode=opmode)
    nd = lat.ndim
    u = [np.asarray(c, dtype=np.float64) for c in u]
    grads = [ops.grad(c, "u") for c in u]            # grads[c][b] = G_b u_c
    laps = [ops.lap(c, "u") for c in u]
    F, ustar = [], []
    for c in range(nd):
        Fc = sum(u[b] * grads[c][b] for b in range(nd)) - nu * laps[c]
        Fp = 0.0 if (k == 0 or F_prev is None) else F_prev[c]
        fc = 0.0 if force is None else force[c]
        us = u[c] - dt * (g * Fc + z * Fp - a * fc)
        F.append(Fc)
        ustar.append(set_dirichlet_walls(us, lat, None if wall is None else wall[c]))
    b = (rho / (a * dt)) * ops.div(ustar)
    phi = ppe.solve(b, lat, family=family)
    gphi = ops.grad(phi, "p")
    unew = [set_dirichlet_walls(ustar[c] - a * (dt / rho) * gphi[c], lat, None if wall is None else wall[c])
            for c in range(nd)]
    if return_parts:
        return unew, phi, F, dict(ustar=ustar, b=b)
    return unew, phi, F
