"""Seeded synthetic inputs (manufactured fields) shared by tests and the bench.

This module holds no arithmetic of the method itself: it only evaluates the
closed-form manufactured fields (and, for the time-dependent workload, the
exact forcing obtained by differentiating them analytically).  Both the GPU
path and the oracle receive the same arrays from here.

All generators use ``numpy.random.default_rng(seed)`` and draw in the order
documented in each function.  Arrays are float64 with numpy shape
[z][y][x] (x fastest); lattice points are x_j = j dx.
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def grid(n, dx):
    """Coordinate arrays (numpy order) for a lattice with n = (nx, ny[, nz])."""
    axes = [np.arange(k) * dx for k in n]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")
    return list(reversed(mesh))            # [x, y(, z)] each with numpy shape


def poly_trig_2d(n, seed: int, dx: float | None = None) -> np.ndarray:
    """Cubic polynomial + 8 terms a_i sin(k_i x + phi_i) cos(l_i y + psi_i).

    Draw order: 10 coefficients c_ab ~ N(0,1) for a + b <= 3 in lexicographic
    (a, b); then per term i: a_i ~ N(0,1), K_i ~ U{1..4}, L_i ~ U{1..4},
    phi_i ~ U(0, 2pi), psi_i ~ U(0, 2pi); k_i = pi K_i, l_i = pi L_i.
    n is an int (n x n lattice) or (nx, ny); dx = 1/(n-1) unless given.
    """
    nx, ny = (n, n) if np.isscalar(n) else n
    dx = 1.0 / (nx - 1) if dx is None else dx
    x = (np.arange(nx) * dx)[None, :]        # separable factors, broadcast over [y][x]
    y = (np.arange(ny) * dx)[:, None]
    rng = np.random.default_rng(seed)
    f = np.zeros((ny, nx))
    for a in range(4):
        for b in range(4 - a):
            f += rng.standard_normal() * x ** a * y ** b
    for _ in range(8):
        amp = rng.standard_normal()
        K = rng.integers(1, 5)
        L = rng.integers(1, 5)
        ph = rng.uniform(0.0, TWO_PI)
        ps = rng.uniform(0.0, TWO_PI)
        f += amp * np.sin(np.pi * K * x + ph) * np.cos(np.pi * L * y + ps)
    return f


def random_field(shape, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) values (unstructured input for operator tests)."""
    return np.random.default_rng(seed).standard_normal(shape)


class DecayingVortexFlow:
    """Manufactured divergence-free 2D flow with known pressure and forcing.

    psi = exp(-t) s sum_{i=1..8} a_i sin(k_i x + phi_i) sin(l_i y + psi_i)
    (seed_u; per term draw a_i ~ N(0,1), K_i ~ U{1..4}, L_i ~ U{1..4},
    phi_i, psi_i ~ U(0, 2pi); k = pi K, l = pi L), u = d psi/dy,
    v = -d psi/dx, with s chosen so that max |u(., 0)| = 1 on the lattice.
    p = exp(-t) sum_{j=1..4} b_j cos(m_j pi x) cos(n_j pi y) (seed_p; per term
    b ~ N(0,1), m ~ U{1..4}, n ~ U{1..4}); homogeneous Neumann on [0,1]^2.
    The forcing f = du/dt + (u . grad) u + grad p / rho - nu lap u makes this
    the exact solution of the incompressible Navier-Stokes equations.
    """

    def __init__(self, n: int, nu: float, rho: float = 1.0, seed_u: int = 10, seed_p: int = 11):
        self.n, self.nu, self.rho = n, nu, rho
        self.dx = 1.0 / (n - 1)
        rng = np.random.default_rng(seed_u)
        self.terms = []
        for _ in range(8):
            a = rng.standard_normal()
            K = rng.integers(1, 5)
            L = rng.integers(1, 5)
            ph = rng.uniform(0.0, TWO_PI)
            ps = rng.uniform(0.0, TWO_PI)
            self.terms.append((a, np.pi * K, np.pi * L, ph, ps))
        rng = np.random.default_rng(seed_p)
        self.pterms = []
        for _ in range(4):
            b = rng.standard_normal()
            m = rng.integers(1, 5)
            nn = rng.integers(1, 5)
            self.pterms.append((b, np.pi * m, np.pi * nn))
        self.x, self.y = grid((n, n), self.dx)
        self.s = 1.0
        u0, v0 = self.velocity(0.0)
        self.s = 1.0 / np.sqrt(np.max(u0 ** 2 + v0 ** 2))

    def _sum(self, t, which):
        x, y = self.x, self.y
        out = np.zeros_like(x)
        for a, k, l, ph, ps in self.terms:
            sx, cx = np.sin(k * x + ph), np.cos(k * x + ph)
            sy, cy = np.sin(l * y + ps), np.cos(l * y + ps)
            out += which(a, k, l, sx, cx, sy, cy)
        return np.exp(-t) * self.s * out

    def velocity(self, t):
        u = self._sum(t, lambda a, k, l, sx, cx, sy, cy: a * l * sx * cy)
        v = self._sum(t, lambda a, k, l, sx, cx, sy, cy: -a * k * cx * sy)
        return u, v

    def pressure(self, t):
        x, y = self.x, self.y
        p = np.zeros_like(x)
        for b, m, nn in self.pterms:
            p += b * np.cos(m * x) * np.cos(nn * y)
        return np.exp(-t) * p

    def force_parts(self):
        """(A, B) with force(t) = exp(-t) A + exp(-2t) B: the linear terms
        (du/dt, grad p, viscous) decay like exp(-t), the advection like exp(-2t)."""
        fa0 = self.force(0.0)
        fa1 = self.force(1.0)
        e1, e2 = np.exp(-1.0), np.exp(-2.0)
        A = [(f1 - e2 * f0) / (e1 - e2) for f0, f1 in zip(fa0, fa1)]
        B = [f0 - a for f0, a in zip(fa0, A)]
        return A, B

    def force(self, t):
        x, y = self.x, self.y
        u, v = self.velocity(t)
        ux = self._sum(t, lambda a, k, l, sx, cx, sy, cy: a * l * k * cx * cy)
        uy = self._sum(t, lambda a, k, l, sx, cx, sy, cy: -a * l * l * sx * sy)
        vx = self._sum(t, lambda a, k, l, sx, cx, sy, cy: a * k * k * sx * sy)
        vy = self._sum(t, lambda a, k, l, sx, cx, sy, cy: -a * k * l * cx * cy)
        lapu = self._sum(t, lambda a, k, l, sx, cx, sy, cy: -(k * k + l * l) * a * l * sx * cy)
        lapv = self._sum(t, lambda a, k, l, sx, cx, sy, cy: (k * k + l * l) * a * k * cx * sy)
        px = np.zeros_like(x)
        py = np.zeros_like(x)
        for b, m, nn in self.pterms:
            px += -b * m * np.sin(m * x) * np.cos(nn * y)
            py += -b * nn * np.cos(m * x) * np.sin(nn * y)
        px *= np.exp(-t)
        py *= np.exp(-t)
        fx = -u + u * ux + v * uy + px / self.rho - self.nu * lapu
        fy = -v + u * vx + v * vy + py / self.rho - self.nu * lapv
        return fx, fy


class ChannelFlow3D:
    """Manufactured divergence-free 3D channel field, walls at y = 0 and y = 1.

    u = (dpsi1/dy, -dpsi1/dx, 0) + (0, -dpsi2/dz, dpsi2/dy) with
    psi_q = y^2 (1-y)^2 sum_{i=1..8} a_i sin(2 pi K_i x / Lx + phi_i) cos(2 pi M_i z / Lz + chi_i)
    (seeds seed1, seed2; per term a ~ N(0,1), K ~ U{1..4}, M ~ U{1..4},
    phi, chi ~ U(0, 2pi)), scaled so that max |u| = 1 on the lattice.
    The lattice is n = (nx, ny, nz) with dx = 1/(ny - 1), Lx = nx dx, Lz = nz dx.
    """

    def __init__(self, n, seed1: int = 20, seed2: int = 21):
        self.n = tuple(n)
        nx, ny, nz = self.n
        self.dx = dx = 1.0 / (ny - 1)
        Lx, Lz = nx * dx, nz * dx
        # separable factors broadcast over [z][y][x]
        x = (np.arange(nx) * dx)[None, None, :]
        y = (np.arange(ny) * dx)[None, :, None]
        z = (np.arange(nz) * dx)[:, None, None]
        comps = [np.zeros((nz, ny, nx)) for _ in range(3)]
        Y = y ** 2 * (1 - y) ** 2
        dY = 2 * y * (1 - y) ** 2 - 2 * y ** 2 * (1 - y)
        for q, seed in enumerate((seed1, seed2)):
            rng = np.random.default_rng(seed)
            for _ in range(8):
                a = rng.standard_normal()
                K = rng.integers(1, 5)
                M = rng.integers(1, 5)
                ph = rng.uniform(0.0, TWO_PI)
                ch = rng.uniform(0.0, TWO_PI)
                kx, kz = TWO_PI * K / Lx, TWO_PI * M / Lz
                X, Z = np.sin(kx * x + ph), np.cos(kz * z + ch)
                dX, dZ = kx * np.cos(kx * x + ph), -kz * np.sin(kz * z + ch)
                if q == 0:      # psi1: (dpsi/dy, -dpsi/dx, 0)
                    comps[0] += a * dY * X * Z
                    comps[1] += -a * Y * dX * Z
                else:           # psi2: (0, -dpsi/dz, dpsi/dy)
                    comps[1] += -a * Y * X * dZ
                    comps[2] += a * dY * X * Z
        s = 1.0 / np.sqrt(np.max(comps[0] ** 2 + comps[1] ** 2 + comps[2] ** 2))
        self.u = [c * s for c in comps]


def gaussian_vortex(n, dx, t, alpha=100.0, x0=0.5, y0=0.5, cx=1.0, cy=0.5):
    """The convected Gaussian of the vortex-convection workload: the initial
    field exp(-alpha r^2) about (x0, y0) translated by (cx t, cy t) (the exact
    solution of linear advection with that velocity).  n = (nx, ny)."""
    nx, ny = n
    x = (np.arange(nx) * dx)[None, :]
    y = (np.arange(ny) * dx)[:, None]
    return np.exp(-alpha * ((x - (x0 + cx * t)) ** 2 + (y - (y0 + cy * t)) ** 2))
