"""Pins of the oracle's FC(Gram) tables (no GPU).

The paper prints no FC(Gram) table, so the tables are pinned by what the
construction fixes: orthonormality of the Gram basis, the fit residuals of the
blend-to-zero continuations (re-evaluated here from the stored trigonometric
coefficients), agreement with an independent least-squares solve (Householder
QR instead of the SVD pseudo-inverse), and the optimality conditions of the
Neumann least-squares problem.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import fcgram


@pytest.fixture(scope="module")
def built():
    return fcgram.build()


def test_committed_table_matches_fresh_build(built, fc_tables):
    tabs, _ = built
    for name in ("Q", "A", "M_D", "M_N"):
        assert np.array_equal(getattr(tabs, name), getattr(fc_tables, name)), name


def test_gram_basis_orthonormal_and_reproduces_vandermonde(built):
    _, mo = built
    Q, R, V = mo["Q"], mo["R"], mo["V"]
    d = Q.rows
    with mp.workdps(64):
        err_orth = max(abs((Q.T * Q)[i, j] - (1 if i == j else 0)) for i in range(d) for j in range(d))
        err_qr = max(abs((Q * R)[i, j] - V[i, j]) for i in range(d) for j in range(d))
        assert all(R[i, i] > 0 for i in range(d))
        assert all(abs(R[i, j]) == 0 for i in range(d) for j in range(i))
    assert err_orth < 1e-60 and err_qr < 1e-55
    tabs, _ = built
    assert np.max(np.abs(tabs.Q.T @ tabs.Q - np.eye(d))) < 1e-15


def test_gram_polynomials_interpolate_columns_of_Q(built):
    _, mo = built
    d = mo["Q"].rows
    with mp.workdps(64):
        for m in range(d):
            for j in range(d):
                val = fcgram.gram_poly(mo["Rinv"], m, mp.mpf(j - (d - 1)))
                assert abs(val - mo["Q"][j, m]) < 1e-55


def test_continuation_fit_residuals(built):
    """g_m matches P_m on the oversampled matching set and vanishes on the zero set."""
    tabs, mo = built
    p = tabs.params
    with mp.workdps(64):
        for m in range(p["d"]):
            coef = mo["coefs"][m]

            def g(x):
                return mp.fsum(a * b for a, b in zip(coef, fcgram.trig_row(x, p["K"], mo["T"])))
            # re-evaluate on a grid finer than the fitting grid (midpoints)
            em = max(abs(g(x + mp.mpf(1) / 40) - fcgram.gram_poly(mo["Rinv"], m, x + mp.mpf(1) / 40))
                     for x in mo["match"][:-1])
            ez = max(abs(g(x + mp.mpf(1) / 40)) for x in mo["zero"][:-1])
            assert em < 2e-15 and ez < 2e-15, (m, em, ez)
            # A holds g_m at the integer continuation points
            for i in range(p["C"]):
                assert abs(g(mp.mpf(i + 1)) - mo["A"][i, m]) < 1e-50


def test_continuation_agrees_with_independent_qr_least_squares(built):
    """Solve the same least-squares fit with Householder QR (mpmath.qr_solve)."""
    tabs, mo = built
    p = tabs.params
    with mp.workdps(64):
        rows = [fcgram.trig_row(x, p["K"], mo["T"]) for x in mo["match"] + mo["zero"]]
        Amat = mp.matrix(rows)
        for m in (0, 2, 4):
            rhs = mp.matrix([fcgram.gram_poly(mo["Rinv"], m, x) for x in mo["match"]]
                            + [0] * len(mo["zero"]))
            coef, _ = mp.qr_solve(Amat, rhs)
            for i in range(p["C"]):
                gi = mp.fsum(a * b for a, b in zip(coef, fcgram.trig_row(mp.mpf(i + 1), p["K"], mo["T"])))
                assert abs(gi - mo["A"][i, m]) < 1e-30 * max(1, abs(gi))


def test_neumann_map_is_the_least_squares_solution(built):
    """Normal equations of [Q; delta^T] c = [f; 0] hold for the stored G_N,
    and Neumann-compatible data (P'(0) = 0) is interpolated exactly."""
    tabs, mo = built
    d = tabs.params["d"]
    with mp.workdps(64):
        aug = mp.matrix(d + 1, d)
        for i in range(d):
            for m in range(d):
                aug[i, m] = mo["Q"][i, m]
        for m in range(d):
            aug[d, m] = mo["Rinv"][1, m]
        rng = np.random.default_rng(5)
        for _ in range(3):
            f = mp.matrix([mp.mpf(float(v)) for v in rng.standard_normal(d)])
            c = mo["G_N"] * f
            rhs = mp.matrix(d + 1, 1)
            for i in range(d):
                rhs[i] = f[i]
            r = aug * c - rhs
            ne = aug.T * r
            assert max(abs(ne[i]) for i in range(d)) < 1e-55
        # Neumann-compatible polynomial: p(xi) = 1 + 0*xi + 0.3 xi^2 - 0.05 xi^3 + 0.01 xi^4
        xi = [mp.mpf(j - (d - 1)) for j in range(d)]
        f = mp.matrix([1 + mp.mpf("0.3") * x ** 2 - mp.mpf("0.05") * x ** 3 + mp.mpf("0.01") * x ** 4 for x in xi])
        cN = mo["G_N"] * f
        cD = mo["Q"].T * f
        assert max(abs(cN[i] - cD[i]) for i in range(d)) < 1e-55
    # the FP64 maps agree on such data
    fv = np.array([float(v) for v in f])
    assert np.max(np.abs(tabs.M_N @ fv - tabs.M_D @ fv)) < 1e-11


def test_table_file_roundtrip(tmp_path, fc_tables):
    p = tmp_path / "t.txt"
    fcgram.write_table(fc_tables, str(p))
    back = fcgram.read_table(str(p))
    for name in ("Q", "A", "M_D", "M_N"):
        assert np.array_equal(getattr(back, name), getattr(fc_tables, name))
