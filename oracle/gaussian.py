"""High-order Gaussian SPH kernels (oracle side).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

Sec. "High-order Gaussian kernel functions" and the appendix deriving the 8th
order kernel: the kernel of order 2n is the base Gaussian times an even
polynomial whose coefficients remove the even moments 2 .. 2(n-1),

    W_2n(q) = (1 / (pi^(d/2) h^d)) P_n(q^2) exp(-q^2),   P_n(s) = sum_{m<n} A_m s^m,

with sum_m A_m I_{m+j} = delta_{j0} (j = 0 .. n-1), I_k the k-th even moment
of the d-dimensional base Gaussian normalised to unit integral: I_k = k! in
2D (the appendix) and Gamma(k + 3/2) / Gamma(3/2) in 3D (the same
construction in three dimensions).  The system is solved here in exact
rational arithmetic.  Readings:
* G10: the coefficients printed in the kernel section violate the moment
  conditions of the appendix's construction; the kernel here is the solution
  of those conditions (5 - 10 q^2 + 5 q^4 - 5 q^6 / 6 + q^8 / 24).  G4, G6 and
  G8 agree with the printed / appendix forms.
* h = 8 dx as printed; the support is infinite, so on a periodic (extended)
  lattice every lattice offset is a tap, sampled at its minimum-image
  displacement per axis (eq. circularConv); an offset of exactly half a
  period along an axis has two images at equal distance, and its weight is
  the average over them (zero for the gradient along that axis).

Closed forms with s = q^2, F(s) = P(s) exp(-s) / (pi^(d/2) h^d):
    W      = F(s)
    grad W = x (2 / h^2) F'(s),            F'(s)  = (P' - P) exp(-s) / (pi^(d/2) h^d)
    lap W  = (4 s F''(s) + 2 d F'(s)) / h^2,  F''(s) = (P'' - 2 P' + P) exp(-s) / (pi^(d/2) h^d)
(d/dr = (2 r / h^2) d/ds; the d-dimensional Laplacian of a radial function is
W'' + (d - 1) W' / r).

Parity: pinned in ``tests/test_oracle_gaussian.py`` by the appendix's G8
coefficients (golden fixture), the closed forms G4 = 2 - q^2, G6 = 3 - 3 q^2 +
q^4 / 2, the moment conditions by independent numerical quadrature, the
derivative closed forms by numerical differentiation of W, brute-force pair
sums with explicit minimum image, and 4th-order convergence of the G4
operators on eq. testFun10 with the paper's own FC.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np

ORDERS = (2, 4, 6, 8, 10)


def moment(k: int, ndim: int) -> Fraction:
    """I_k = int q^(2k) W_G2 dV / int W_G2 dV of the unit-integral base Gaussian."""
    if ndim == 2:
        return Fraction(math.factorial(k))
    if ndim == 3:
        out = Fraction(1)
        for i in range(1, k + 1):
            out *= Fraction(2 * i + 1, 2)         # Gamma(i + 3/2) / Gamma(i + 1/2)
        return out
    raise ValueError("ndim must be 2 or 3")


def coefficients(order: int, ndim: int = 2) -> list:
    """A_0 .. A_{n-1} (exact rationals) of the order-2n kernel: the solution of
    sum_m A_m I_{m+j} = delta_{j0}, j = 0 .. n-1 (Gaussian elimination over
    the rationals)."""
    if order not in ORDERS:
        raise ValueError(f"order must be one of {ORDERS}")
    n = order // 2
    M = [[moment(m + j, ndim) for m in range(n)] + [Fraction(1 if j == 0 else 0)] for j in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [a - f * b for a, b in zip(M[r], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


def _poly(A, s, deriv=0):
    """P^(deriv)(s) for P(s) = sum A_m s^m (float coefficients)."""
    out = np.zeros_like(np.asarray(s, dtype=np.float64))
    for m, a in enumerate(A):
        if m < deriv:
            continue
        c = float(a) * math.perm(m, deriv)
        out = out + c * np.asarray(s, dtype=np.float64) ** (m - deriv)
    return out


class GaussianKernel:
    """W_2n on d dimensions with smoothing length h."""

    def __init__(self, order: int, ndim: int, h: float):
        self.order, self.ndim, self.h = order, ndim, h
        self.A = coefficients(order, ndim)
        self.norm = 1.0 / (math.pi ** (ndim / 2.0) * h ** ndim)

    def W(self, r):
        s = (np.asarray(r, dtype=np.float64) / self.h) ** 2
        return self.norm * _poly(self.A, s) * np.exp(-s)

    def dF(self, s):
        return self.norm * (_poly(self.A, s, 1) - _poly(self.A, s)) * np.exp(-s)

    def d2F(self, s):
        return self.norm * (_poly(self.A, s, 2) - 2 * _poly(self.A, s, 1) + _poly(self.A, s)) * np.exp(-s)

    def gradW(self, xvec):
        """Gradient at displacement xvec (last axis = components)."""
        xvec = np.asarray(xvec, dtype=np.float64)
        s = np.sum(xvec ** 2, axis=-1) / self.h ** 2
        return (2.0 / self.h ** 2) * self.dF(s)[..., None] * xvec

    def lapW(self, r):
        s = (np.asarray(r, dtype=np.float64) / self.h) ** 2
        return (4.0 * s * self.d2F(s) + 2.0 * self.ndim * self.dF(s)) / self.h ** 2


def min_image_offsets(E: int) -> list:
    """Per-axis lattice offsets of a period-E axis with their minimum-image
    displacements (in lattice units): offset s in (-E/2, E/2]; s = E/2 (even
    E) has the two images +E/2 and -E/2."""
    out = []
    for s in range(-((E - 1) // 2), E // 2 + 1):
        imgs = (s, -s) if 2 * s == E else (s,)
        out.append((s, imgs))
    return out


def taps(kernel: GaussianKernel, dx: float, ext) -> list:
    """(offset, w_grad[ndim], w_lap) for every lattice offset of the extended
    lattice with periods ext (lattice order): dV times the kernel derivatives
    at the minimum-image displacement, averaged over the images of an
    offset at exactly half a period."""
    nd = len(ext)
    dV = dx ** nd
    per_axis = [min_image_offsets(E) for E in ext]
    out = []
    for combo in itertools.product(*per_axis):
        s = tuple(c[0] for c in combo)
        images = list(itertools.product(*[c[1] for c in combo]))
        g = np.zeros(nd)
        lap = 0.0
        for img in images:
            xv = np.array(img, dtype=np.float64) * dx
            g += kernel.gradW(xv) * dV
            lap += float(kernel.lapW(np.sqrt(np.sum(xv * xv)))) * dV
        out.append((s, g / len(images), lap / len(images)))
    return out
