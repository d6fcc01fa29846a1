"""SPH kernel closed forms and lattice taps (oracle side).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

The operators of eq. SPHConV / eq. circularConv weight f_j by the kernel
gradient at x_i - x_j times the particle volume.  The kernel used for the hot
path is Wendland C2 (not one of the paper's Gaussians; the paper's G4..G10 are
listed in Sec. "High-order Gaussian kernel functions" and its appendix).

Wendland C2 with q = r/h, s = 1 - q/2, support q < 2:
    W      = alpha s^4 (1 + 2q)
    grad W = -(5 alpha / h^2) s^3 x                  (vector x = x_i - x_j)
    lap  W = -(5 alpha / h^2) s^2 (2 - 5q/2)  in 2D
           = -(5 alpha / h^2) s^2 (3 - 3q)    in 3D
    alpha  = 7 / (4 pi h^2) in 2D, 21 / (16 pi h^3) in 3D
These follow from differentiating W (dW/dq = -5 alpha q s^3); they are pinned in
tests by numerical differentiation of W and by the normalisation integral.

Taps: every integer lattice offset s with |s| dx < 2h.  For offset s
(= i - j, so x_i - x_j = s dx) the weights are
    w_a(s) = dV * d/dx_a W (s dx)      w_L(s) = dV * lap W (s dx)
with dV = dx^ndim (the particle volume of eq. circularConv).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def wendland_alpha(h: float, ndim: int) -> float:
    if ndim == 2:
        return 7.0 / (4.0 * math.pi * h * h)
    if ndim == 3:
        return 21.0 / (16.0 * math.pi * h ** 3)
    raise ValueError("ndim must be 2 or 3")


def wendland_W(r, h: float, ndim: int):
    q = np.asarray(r, dtype=np.float64) / h
    s = np.clip(1.0 - q / 2.0, 0.0, None)
    return wendland_alpha(h, ndim) * s ** 4 * (1.0 + 2.0 * q)


def wendland_gradW(xvec, h: float, ndim: int):
    """Gradient of W at displacement xvec (last axis = components)."""
    xvec = np.asarray(xvec, dtype=np.float64)
    r = np.sqrt(np.sum(xvec ** 2, axis=-1))
    q = r / h
    s = np.clip(1.0 - q / 2.0, 0.0, None)
    fac = -5.0 * wendland_alpha(h, ndim) / h ** 2 * s ** 3
    return fac[..., None] * xvec


def wendland_lapW(r, h: float, ndim: int):
    q = np.asarray(r, dtype=np.float64) / h
    s = np.clip(1.0 - q / 2.0, 0.0, None)
    pre = -5.0 * wendland_alpha(h, ndim) / h ** 2 * s ** 2
    if ndim == 2:
        return np.where(q < 2.0, pre * (2.0 - 2.5 * q), 0.0)
    return np.where(q < 2.0, pre * (3.0 - 3.0 * q), 0.0)


def taps(ndim: int, dx: float, h_over_dx: float):
    """List of (offset, w_grad[ndim], w_lap) for every offset inside the support.

    Offsets are tuples in lattice order (sx, sy[, sz]).
    """
    h = h_over_dx * dx
    rad = int(math.floor(2.0 * h_over_dx))
    dV = dx ** ndim
    out = []
    for s in itertools.product(range(-rad, rad + 1), repeat=ndim):
        r2 = sum(c * c for c in s)
        if math.sqrt(r2) >= 2.0 * h_over_dx:      # |s| dx < 2h
            continue
        xv = np.array(s, dtype=np.float64) * dx
        g = wendland_gradW(xv, h, ndim) * dV
        lap = float(wendland_lapW(math.sqrt(r2) * dx, h, ndim)) * dV
        out.append((tuple(s), g.astype(np.float64), lap))
    return out
