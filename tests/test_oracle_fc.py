"""Pins of the oracle's FC apply (no GPU).

P-FC1  physical values are copied unchanged (bitwise).
P-FC5  the extension of degree < d polynomials is smooth across the walls: a
       spectral (ik) derivative of the periodic extension reproduces the
       analytic derivative at the physical points.
P-FC7  for the paper's example f = e^y sin(5y) + 0.5 y^3 (Sec. "Step 2"
       figure) the spectral derivative of the extension converges at >= 4th
       order under refinement; the 2D test function (eq. testFun10) is a
       degree-4 polynomial in y and is reproduced to round-off.
Mirror: extending the reversed line gives the reversed extension (pins the
       low-wall index mapping).
Order : in 2D the result does not depend on the axis order.
"""
import numpy as np
import pytest

from oracle import fc


def spectral_derivative(e, dx):
    k = 2 * np.pi * np.fft.fftfreq(len(e), d=dx)
    return np.real(np.fft.ifft(1j * k * np.fft.fft(e)))


def test_physical_values_copied_bitwise(fc_tables):
    rng = np.random.default_rng(0)
    f = rng.standard_normal((40, 33))
    e = fc.extend(f, (True, True), (("D", "N"), ("N", "D")), fc_tables)
    assert e.shape == (40 + 25, 33 + 25)
    assert np.array_equal(e[:40, :33], f)


@pytest.mark.parametrize("n", [32, 64, 128, 256, 512, 1024])
@pytest.mark.parametrize("bc", ["D", "N"])
def test_polynomial_extension_is_smooth(fc_tables, n, bc):
    y = np.linspace(0.0, 1.0, n)
    dx = 1.0 / (n - 1)
    if bc == "D":
        f = 1 + 2 * y - 3 * y ** 2 + y ** 3 + 0.5 * y ** 4
        fp = 2 - 6 * y + 3 * y ** 2 + 2 * y ** 3
    else:   # zero slope at both walls: f' = y^2 (1-y)^2 ...
        f = y ** 3 / 3 - y ** 4 / 2 + y ** 5 / 5
        fp = y ** 2 * (1 - y) ** 2
        # degree 5 > d-1: only Neumann-compatible and smooth, not exact
    M = fc_tables.M(bc)
    e = fc.extend_line_axis(f, 0, M, M)
    d = spectral_derivative(e, dx)[:n]
    err = np.max(np.abs(d - fp)) / np.max(np.abs(fp))
    if bc == "D":
        assert err < 1e-11 * n, err
    else:
        assert err < 5e-3 * (32.0 / n) ** 4 + 1e-11 * n, err


def _order(errs, ns):
    return [np.log(errs[i] / errs[i + 1]) / np.log((ns[i + 1] - 1) / (ns[i] - 1)) for i in range(len(ns) - 1)]


def test_example_function_converges_fourth_order(fc_tables):
    ns = [32, 64, 128, 256]
    errs = []
    for n in ns:
        y = np.linspace(0.0, 1.0, n)
        f = np.exp(y) * np.sin(5 * y) + 0.5 * y ** 3
        fp = np.exp(y) * np.sin(5 * y) + 5 * np.exp(y) * np.cos(5 * y) + 1.5 * y ** 2
        e = fc.extend_line_axis(f, 0, fc_tables.M_D, fc_tables.M_D)
        errs.append(np.max(np.abs(spectral_derivative(e, 1.0 / (n - 1))[:n] - fp)))
    orders = _order(errs, ns)
    assert min(orders) >= 4.0, (errs, orders)


def test_test_function_2d_is_reproduced(fc_tables):
    """eq. testFun10: periodic in x, walls in y.  Along y it is a polynomial of
    degree 4 < d, which the Gram projection reproduces, so the spectral y
    derivative of its extension is exact up to round-off at every size."""
    ns = [32, 64, 128, 256]
    errs = []
    for n in ns:
        dy = 1.0 / (n - 1)
        y = np.arange(n) * dy
        x = np.arange(16) / 16.0
        X, Y = np.meshgrid(x, y, indexing="xy")
        f = np.sin(2 * np.pi * X) * Y * (1 - Y) + 0.5 * np.cos(4 * np.pi * X) * Y ** 2 * (1 - Y) ** 2
        fy = np.sin(2 * np.pi * X) * (1 - 2 * Y) + 0.5 * np.cos(4 * np.pi * X) * (2 * Y * (1 - Y) ** 2 - 2 * Y ** 2 * (1 - Y))
        e = fc.extend(f, (False, True), (None, ("D", "D")), fc_tables)
        k = 2 * np.pi * np.fft.fftfreq(e.shape[0], d=dy)
        d = np.real(np.fft.ifft(1j * k[:, None] * np.fft.fft(e, axis=0), axis=0))[:n]
        errs.append(np.max(np.abs(d - fy)))
    assert max(errs) < 1e-9, errs


def test_mirror_symmetry_of_low_and_high_walls(fc_tables):
    rng = np.random.default_rng(1)
    f = rng.standard_normal(50)
    for lo, hi in (("D", "D"), ("D", "N"), ("N", "D")):
        e = fc.extend_line_axis(f, 0, fc_tables.M(lo), fc_tables.M(hi))
        er = fc.extend_line_axis(f[::-1], 0, fc_tables.M(hi), fc_tables.M(lo))
        # reversing the periodic line about index 0's image: e_rev[j] = e[(n-1-j) mod E]
        n, E = len(f), len(e)
        idx = (n - 1 - np.arange(E)) % E
        assert np.allclose(er, e[idx], rtol=0, atol=1e-12)


def test_axis_order_independence(fc_tables):
    rng = np.random.default_rng(2)
    f = rng.standard_normal((30, 41))
    bcs = (("D", "N"), ("N", "N"))
    e1 = fc.extend(f, (True, True), bcs, fc_tables, order=(0, 1))
    e2 = fc.extend(f, (True, True), bcs, fc_tables, order=(1, 0))
    assert np.max(np.abs(e1 - e2)) < 1e-9 * np.max(np.abs(e1))
