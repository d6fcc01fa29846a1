"""Spectral SPH operators as circular convolutions (oracle side).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

Sec. "Linear and circular convolution", eq. circularConv: on the FC-extended
periodic lattice the derivative at particle i is
    (G_a f)_i = sum_j f_j d_a W((x_i - x_j) mod L) dV  =  sum_s w_a(s) e[(i - s) mod n_ext]
with the minimum-image separation (s = i - j); the Laplacian uses the kernel
Laplacian in the same way (reading: kernel-weighted Laplacian, f convolved with
dV lap W).  Eq. final_dft_gradient computes the same circular convolution by
the convolution theorem; that equality is the discrete convolution theorem,
so the oracle evaluates the definition directly: a tap sum over the compact
Wendland support, with ``np.roll`` providing the periodic index (i - s) mod n.
Outputs are restricted to the physical lattice (wall points included).

``mode='fft'`` computes the same math with scipy.fft (the convolution theorem,
symbols = DFT of the sampled, corner-wrapped taps); it exists only as the timed
CPU baseline and is cross-checked against the direct mode in tests.

Kernels: Wendland C2 (compact, ``oracle.kernels``) or the Gaussian family
(``oracle.gaussian``: infinite support, every offset of the extended lattice
at its minimum image).

Parity: pinned by brute-force O(E^2) pair sums with explicit minimum image
(P-OP1), the Fourier eigen-test (P-OP2), closed-form lattice sums at interior
points (P-OP3) and antisymmetry (P-OP4) in ``tests/test_oracle_operators.py``;
with the Gaussian kernels by pair sums and 4th-order convergence in
``tests/test_oracle_gaussian.py``.
"""
from __future__ import annotations

import functools

import numpy as np

from . import fc as fcmod
from . import kernels


def conv_direct(e: np.ndarray, tap_list) -> np.ndarray:
    """out[i] = sum_s w(s) e[(i - s) mod n] over lattice-order offsets s."""
    ndim = e.ndim
    out = np.zeros_like(e, dtype=np.float64)
    for s, w in tap_list:
        if w == 0.0:
            continue
        shift = tuple(reversed(s))                 # numpy axis order (.., y, x)
        out += w * np.roll(e, shift=shift, axis=tuple(range(ndim)))
    return out


def corner_wrapped_kernel(shape_np, tap_list) -> np.ndarray:
    """Sampled kernel array with offset s stored at index s mod shape (eq. circularConv,
    kernel wrapped to the corners of the extended grid)."""
    k = np.zeros(shape_np, dtype=np.float64)
    for s, w in tap_list:
        idx = tuple(c % n for c, n in zip(reversed(s), shape_np))
        k[idx] += w
    return k


def conv_fft(e: np.ndarray, tap_list, workers: int = -1) -> np.ndarray:
    import scipy.fft as sfft
    ker = corner_wrapped_kernel(e.shape, tap_list)
    return sfft.irfftn(sfft.rfftn(e, workers=workers) * sfft.rfftn(ker, workers=workers),
                       s=e.shape, workers=workers)


@functools.lru_cache(maxsize=8)
def _gaussian_taps(order, ndim, h_over_dx, dx, ext):
    """The Gaussian tap list of one lattice, built once (it is the same for
    every operator call on that lattice)."""
    from . import gaussian
    return gaussian.taps(gaussian.GaussianKernel(order, ndim, h_over_dx * dx), dx, ext)


class Operators:
    """Gradient / divergence / Laplacian on one lattice.

    lat: an ``oracle.lattice.Lattice``;  tables: FC(Gram) tables.
    """

    def __init__(self, lat, tables, mode: str = "direct"):
        self.lat = lat
        self.tables = tables
        self.mode = mode
        if lat.kernel == "wendland_c2":
            tl = kernels.taps(lat.ndim, lat.dx, lat.h_over_dx)
        else:
            # Gaussian family: every offset of the extended lattice (minimum image)
            tl = _gaussian_taps(int(lat.kernel[1:]), lat.ndim, lat.h_over_dx, lat.dx, tuple(lat.ext))
        self.grad_taps = [[(s, float(g[a])) for s, g, _ in tl] for a in range(lat.ndim)]
        self.lap_taps = [(s, lap) for s, _, lap in tl]

    def _conv(self, e, tl):
        if self.mode == "direct":
            return conv_direct(e, tl)
        return conv_fft(e, tl)

    def extend(self, f, field: str):
        """FC extension with the velocity ('u') or pressure ('p') wall types."""
        bcs = self.lat.vel_bc if field == "u" else self.lat.prs_bc
        return fcmod.extend(f, self.lat.walled, bcs, self.tables)

    def restrict(self, e):
        return fcmod.restrict(e, self.lat.n)

    def grad(self, f, field: str = "u"):
        e = self.extend(f, field)
        return [self.restrict(self._conv(e, self.grad_taps[a])) for a in range(self.lat.ndim)]

    def div(self, us):
        out = None
        for a, u in enumerate(us):
            e = self.extend(u, "u")
            t = self._conv(e, self.grad_taps[a])
            out = t if out is None else out + t
        return self.restrict(out)

    def lap(self, f, field: str = "u"):
        return self.restrict(self._conv(self.extend(f, field), self.lap_taps))
