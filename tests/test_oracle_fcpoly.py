"""Pins of the oracle's tables for the paper's own FC (polynomial fit,
extrapolation, quintic blend; no GPU).

P-PF1 : a constant continues as the same constant: the two blend weights sum
        to one at every continuation point (mirroring and weights consistent).
P-PF2 : the blend weight w_r = M_D[r-1] . 1 is 1 at the first continuation
        point, 0 at the last, decreasing, and mirror symmetric
        (w_r + w_{C+1-r} = 1), which lets one map serve both walls.
P-PF3 : every polynomial q of degree <= p is fitted exactly, so
        M_D[r-1] . q(xi_j) = w_r q(r) (one-sided extrapolation times the
        weight); a degree p+1 polynomial is not reproduced.
P-PF4 : Neumann: data of an even polynomial about the wall satisfy the
        derivative row, so M_N reproduces them as M_D does; for odd data the
        derivative row pulls the fitted slope at the wall towards zero.
P-PF5 : the extended line of the paper's example function e^y sin(5y) +
        0.5 y^3 is smooth enough that its FFT derivative converges at the
        physical points as the lattice is refined (extension 0.25 n; second
        order, measured 1.1e-3, 3.0e-4, 7.8e-5 at n = 65, 129, 257: the blend
        is C^2 at the junctions).
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import fc as ofc
from oracle import fcpoly


@pytest.fixture(scope="module")
def tab():
    return fcpoly.build(d=10, p=5, C=24)


def _xi(d):
    return np.arange(d) - (d - 1.0)


def test_constant_continues_as_constant(tab):
    f = np.full(40, 3.25)
    e = ofc.extend_line_axis(f, 0, tab.M_D, tab.M_D)
    assert np.max(np.abs(e - 3.25)) < 1e-12 * 3.25


def test_blend_weights(tab):
    w = tab.M_D @ np.ones(10)
    C = len(w)
    # FP64 rounding of a 10-term row sum of entries up to max |M|
    tol = 10 * np.finfo(float).eps * np.max(np.abs(tab.M_D))
    assert abs(w[0] - 1) < tol and abs(w[-1]) < tol
    assert np.all(np.diff(w) < 0)
    assert np.max(np.abs(w + w[::-1] - 1)) < tol
    # the same weights multiply the Neumann fit
    assert np.max(np.abs(tab.M_N @ np.ones(10) - w)) < 10 * np.finfo(float).eps * np.max(np.abs(tab.M_N)) + tol
    assert C == 24


@pytest.mark.parametrize("deg", [1, 2, 3, 4, 5])
def test_polynomials_extrapolated_exactly(tab, deg):
    rng = np.random.default_rng(deg)
    c = rng.standard_normal(deg + 1)
    q = lambda x: sum(c[m] * x ** m for m in range(deg + 1))  # noqa: E731
    w = tab.M_D @ np.ones(10)
    r = np.arange(1, 25, dtype=float)
    got = tab.M_D @ q(_xi(10))
    ref = w * q(r)
    assert np.max(np.abs(got - ref)) < 1e-9 * max(1.0, np.max(np.abs(ref)))


def test_degree_above_p_not_reproduced(tab):
    q = _xi(10) ** 6
    w = tab.M_D @ np.ones(10)
    r = np.arange(1, 25, dtype=float)
    assert np.max(np.abs(tab.M_D @ q - w * r ** 6)) > 1.0


def test_neumann_fit(tab):
    w = tab.M_D @ np.ones(10)
    r = np.arange(1, 25, dtype=float)
    even = lambda x: 1.0 + 0.3 * x ** 2 - 0.01 * x ** 4  # noqa: E731
    assert np.max(np.abs(tab.M_N @ even(_xi(10)) - w * even(r))) < 1e-9 * np.max(np.abs(w * even(r)))
    # slope of the fitted polynomial at the wall for data xi: 1 for Dirichlet,
    # pulled towards 0 by the Neumann row
    PD = fcpoly.solution_operator(10, 5, False)
    PN = fcpoly.solution_operator(10, 5, True)
    data = [Fraction(int(x)) for x in _xi(10)]
    sD = sum(PD[1][j] * data[j] for j in range(10))
    sN = sum(PN[1][j] * data[j] for j in range(10))
    assert sD == 1 and 0 <= sN < 1


def test_example_function_spectral_derivative_converges():
    errs = []
    for n in (65, 129, 257):
        dx = 1.0 / (n - 1)
        y = np.arange(n) * dx
        f = np.exp(y) * np.sin(5 * y) + 0.5 * y ** 3
        df = np.exp(y) * (np.sin(5 * y) + 5 * np.cos(5 * y)) + 1.5 * y ** 2
        C = (n - 1) // 4
        t = fcpoly.build(d=10, p=5, C=C)
        e = ofc.extend_line_axis(f, 0, t.M_D, t.M_D)
        E = len(e)
        k = np.fft.fftfreq(E, d=dx) * 2 * np.pi
        de = np.real(np.fft.ifft(1j * k * np.fft.fft(e)))
        errs.append(np.max(np.abs(de[:n] - df)) / np.max(np.abs(df)))
    assert errs[-1] < 1e-3, errs
    assert errs[0] / errs[1] > 3 and errs[1] / errs[2] > 3, errs
