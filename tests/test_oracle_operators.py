"""Pins of the oracle's kernel and operators (no GPU).

Kernel : Wendland C2 is normalised (quadrature of W over its support is 1);
         the closed-form gradient and Laplacian agree with finite differences
         of W; the support holds 21 (2D) / 81 (3D) taps at h/dx = 1.3.
P-OP1  : the direct tap sum equals a brute-force O(E^2) pair sum of
         eq. circularConv with an explicit minimum-image separation, and the
         FFT mode (convolution theorem) agrees.
P-OP2  : a single Fourier mode is an eigenvector, scaled by the closed-form
         trigonometric sum over the taps.
P-OP3  : at interior points the taps never reach the continuation, so
         G_x(1) = 0 exactly and G_x(x) is the lattice first moment, which tends
         to 1 for wide kernels (consistency of the kernel gradient).
P-OP4  : G_a is antisymmetric and L symmetric on periodic lattices.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import kernels, operators
from oracle.lattice import Lattice, walled_box


@pytest.mark.parametrize("ndim", [2, 3])
def test_wendland_normalised(ndim):
    h = 0.7
    if ndim == 2:
        val, _ = integrate.quad(lambda r: 2 * np.pi * r * kernels.wendland_W(r, h, 2), 0, 2 * h)
    else:
        val, _ = integrate.quad(lambda r: 4 * np.pi * r * r * kernels.wendland_W(r, h, 3), 0, 2 * h)
    assert abs(val - 1.0) < 1e-12


@pytest.mark.parametrize("ndim", [2, 3])
def test_wendland_derivatives_match_finite_differences(ndim):
    h = 0.9
    rng = np.random.default_rng(3)
    eps = 1e-5
    for _ in range(20):
        x = rng.uniform(-1.2, 1.2, ndim)
        if np.linalg.norm(x) >= 2 * h - 0.05:
            continue
        W = lambda v: float(kernels.wendland_W(np.linalg.norm(v), h, ndim))
        g = kernels.wendland_gradW(x, h, ndim)
        lap_fd = 0.0
        for a in range(ndim):
            e = np.zeros(ndim)
            e[a] = eps
            gfd = (W(x + e) - W(x - e)) / (2 * eps)
            assert abs(gfd - g[a]) < 1e-7 * (1 + abs(g[a]))
            lap_fd += (W(x + e) - 2 * W(x) + W(x - e)) / eps ** 2
        lap = float(kernels.wendland_lapW(np.linalg.norm(x), h, ndim))
        assert abs(lap_fd - lap) < 1e-4 * (1 + abs(lap))


def test_tap_counts():
    assert len(kernels.taps(2, 0.01, 1.3)) == 21
    assert len(kernels.taps(3, 0.01, 1.3)) == 81


def brute_force(e, dx, h_over_dx, a):
    """O(E^2): sum_j f_j dV d_aW(min-image(x_i - x_j)) for every i; a = axis or 'lap'."""
    shp = e.shape
    nd = e.ndim
    h = h_over_dx * dx
    L = np.array(list(reversed(shp))) * dx        # lattice order
    pts = list(itertools.product(*[range(k) for k in shp]))
    out = np.zeros(shp)
    dV = dx ** nd
    for i in pts:
        xi = np.array(list(reversed(i))) * dx
        acc = 0.0
        for j in pts:
            xj = np.array(list(reversed(j))) * dx
            r = xi - xj
            r = r - L * np.round(r / L)               # nearest periodic image
            rr = math.sqrt(float(np.sum(r * r)))
            if rr >= 2 * h:
                continue
            if a == "lap":
                w = float(kernels.wendland_lapW(rr, h, nd))
            else:
                w = float(kernels.wendland_gradW(r, h, nd)[a])
            acc += e[j] * w * dV
        out[i] = acc
    return out


@pytest.mark.parametrize("shape", [(9, 13), (16, 16), (7, 10, 12)])
def test_direct_sum_equals_brute_force(shape):
    rng = np.random.default_rng(4)
    e = rng.standard_normal(shape)
    nd = len(shape)
    dx = 0.1
    tl = kernels.taps(nd, dx, 1.3)
    for a in list(range(nd)) + ["lap"]:
        if a == "lap":
            taps = [(s, lap) for s, _, lap in tl]
        else:
            taps = [(s, float(g[a])) for s, g, _ in tl]
        ref = brute_force(e, dx, 1.3, a)
        got = operators.conv_direct(e, taps)
        fft = operators.conv_fft(e, taps, workers=1)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(got - ref)) < 1e-13 * scale
        assert np.max(np.abs(fft - ref)) < 1e-13 * scale


def test_fourier_mode_eigen():
    nx, ny = 24, 18
    dx = 1.0 / 20
    tl = kernels.taps(2, dx, 1.3)
    j = np.arange(ny)[:, None]
    i = np.arange(nx)[None, :]
    for kx, ky in ((0, 0), (3, 5), (12, 9), (7, 1)):
        mode = np.exp(2j * np.pi * (kx * i / nx + ky * j / ny))
        for a in (0, 1):
            taps = [(s, float(g[a])) for s, g, _ in tl]
            S = sum(w * np.exp(-2j * np.pi * (kx * s[0] / nx + ky * s[1] / ny)) for s, w in taps)
            got = operators.conv_direct(mode.real, taps) + 1j * operators.conv_direct(mode.imag, taps)
            assert np.max(np.abs(got - S * mode)) < 1e-12 * max(1.0, abs(S))
            assert abs(S.real) < 1e-12 * max(1.0, abs(S))           # odd taps: purely imaginary
        taps = [(s, lap) for s, _, lap in tl]
        SL = sum(w * np.exp(-2j * np.pi * (kx * s[0] / nx + ky * s[1] / ny)) for s, w in taps)
        assert abs(SL.imag) < 1e-9 * abs(SL)                       # even taps: real


def test_interior_moments_and_consistency(fc_tables):
    n = 40
    lat = walled_box((n, n))
    ops = operators.Operators(lat, fc_tables)
    x = np.arange(n) * lat.dx
    X = np.broadcast_to(x[None, :], (n, n)).copy()
    inner = (slice(3, n - 3), slice(3, n - 3))
    gx1 = ops.grad(np.ones((n, n)))[0]
    assert np.max(np.abs(gx1[inner])) < 1e-12
    m1 = ops.grad(X)[0][inner]
    assert np.ptp(m1) < 1e-12
    # the first lattice moment tends to 1 as the kernel widens (the gradient of
    # a linear function is reproduced in the continuum limit of the kernel)
    devs = []
    for hod in (1.3, 2.0, 3.0):
        lat2 = walled_box((40, 40), h_over_dx=hod)
        o2 = operators.Operators(lat2, fc_tables)
        r = int(2 * hod) + 1
        g = o2.grad(X)[0][r:n - r, r:n - r]
        assert np.ptp(g) < 1e-12
        devs.append(abs(1.0 - g[0, 0]))
    assert devs[0] > devs[1] > devs[2] and devs[2] < 1e-4, devs
    assert devs[0] > 0.02          # h/dx = 1.3 leaves a lattice bias in the moment


def test_antisymmetry_and_symmetry():
    lat = Lattice(n=(20, 15), walled=(False, False), dx=0.05)
    ops = operators.Operators(lat, None)
    rng = np.random.default_rng(6)
    f, g = rng.standard_normal((2, 15, 20))
    for a in range(2):
        lhs = np.sum(g * ops.grad(f)[a])
        rhs = -np.sum(ops.grad(g)[a] * f)
        assert abs(lhs - rhs) < 1e-12 * np.sum(np.abs(g * ops.grad(f)[a]))
    assert abs(np.sum(g * ops.lap(f)) - np.sum(ops.lap(g) * f)) < 1e-11 * np.sum(np.abs(g * ops.lap(f)))


def test_direct_and_fft_modes_agree_on_walled_lattice(fc_tables):
    from paper_2606_06247_amd import synth
    lat = walled_box((33, 33), vel_bc=(("D", "N"), ("N", "D")))
    f = synth.poly_trig_2d(33, seed=7)
    o1 = operators.Operators(lat, fc_tables, mode="direct")
    o2 = operators.Operators(lat, fc_tables, mode="fft")
    for a, b in zip(o1.grad(f) + [o1.lap(f)], o2.grad(f) + [o2.lap(f)]):
        assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_wendland_laplacian_does_not_annihilate_constants():
    """The sampled kernel Laplacian of Wendland C2 at h = 1.3 dx sums to
    -0.745 / dx^2 over the lattice instead of 0, so the operator maps a
    constant field to that multiple of it (a property of the kernel at this
    smoothing length; the Gaussian G4 at h = 8 dx sums to nearly 0).  The
    oracle's Laplacian of a constant (FC, corner-wrapped taps, circular
    convolution) equals the brute-force lattice sum of the closed form
    lap W = (alpha / h^2) (1 - q/2)^2 (12.5 q - 10), q = r / h < 2, derived by
    hand from W = alpha (1 - q/2)^4 (2q + 1), alpha = 7 / (4 pi h^2)."""
    import math
    from oracle.lattice import Lattice
    h = 1.3                                    # in units of dx
    alpha = 7.0 / (4.0 * math.pi * h * h)
    brute = 0.0
    for i in range(-3, 4):
        for j in range(-3, 4):
            q = math.hypot(i, j) / h
            if q < 2.0:
                brute += alpha / (h * h) * (1.0 - q / 2.0) ** 2 * (12.5 * q - 10.0)
    assert abs(brute - (-0.74503)) < 1e-4
    n = 40
    lat = Lattice(n=(n, n), walled=(False, False), dx=1.0 / n)
    L = operators.Operators(lat, None, mode="direct").lap(np.ones((n, n)), "u")
    assert np.allclose(L * lat.dx ** 2, brute, rtol=1e-12, atol=0)
    g4 = Lattice(n=(48, 48), walled=(False, False), dx=1.0 / 48, h_over_dx=8.0, kernel="g4")
    L4 = operators.Operators(g4, None, mode="fft").lap(np.ones((48, 48)), "u")
    assert np.max(np.abs(L4)) * g4.dx ** 2 < 1e-3
