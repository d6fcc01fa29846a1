"""FC(Gram) continuation matrices, built in extended precision (oracle side).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``): never imported by the
product path.

What the paper fixes
--------------------
Sec. "Fourier Continuation (FC) Algorithm", closing paragraph: the FC(Gram)
variant projects the wall data onto a Gram polynomial basis and applies
precomputed continuation matrices as matrix-vector products.  The paper defers
the construction to the FC(Gram) literature, so the construction below is a
reading (recorded with its parameters in the table header):

1. Gram basis.  Matching points in grid units with the wall at 0:
   xi_j = j - (d-1), j = 0..d-1.  V[j, m] = xi_j**m, V = Q R (Householder,
   diag(R) > 0).  The Gram polynomials as functions are
   [P_0 .. P_{d-1}](xi) = [1, xi, .., xi^{d-1}] R^{-1}; Q[j, m] = P_m(xi_j).
2. Blend-to-zero continuation of each P_m: a trigonometric polynomial
   g_m(xi) = a_0 + sum_{k=1..K} a_k cos(2 pi k xi / T) + b_k sin(2 pi k xi / T)
   fitted in the least-squares sense to P_m on the oversampled matching
   interval [-(d-1), 0] (step 1/n_os) and to 0 on the oversampled zero
   interval [C+1, C+Z]; period T = d + C + Z + E - 1.  The fit is the exact
   (untruncated) least-squares solution, obtained here through the SVD
   pseudo-inverse at ``dps`` decimal digits.  Because the system has full
   column rank at that precision, the solution is unique and any accurate
   least-squares solver reproduces it.
3. A[i-1, m] = g_m(i), i = 1..C   (C x d).
4. Dirichlet map  M_D = A Q^T, acting on (f_{n-d}, .., f_{n-1}).
5. Neumann map: the paper's Neumann mechanism (eq. FCNeumann) appends one
   derivative row with right-hand side 0 to the least-squares system.  In the
   Gram basis the row is delta_m = P_m'(0) (grid units), the coefficients are
   the least-squares solution of [Q; delta^T] c = [f; 0], i.e.
   c = G_N f with G_N the first d columns of pinv([Q; delta^T]), and
   M_N = A G_N.  The row is unweighted (literal reading of eq. FCNeumann).

Parity: the table values themselves have no published reference ("parity
unpinned" for the raw entries).  They are pinned by invariants in
``tests/test_oracle_fcgram.py``: Q^T Q = I, QR = V, exact reproduction of
degree < d data by the Gram projection, the Neumann map on Neumann-compatible
polynomials, the fit residuals on the matching and zero sets, and agreement
with an independent brute-force least-squares solve.
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass, field

import mpmath as mp
import numpy as np

DEFAULT_PARAMS = dict(d=5, C=25, Z=12, E=25, n_os=20, K=25, dps=64)

TABLE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tables")


@dataclass
class FCGramTables:
    """Continuation tables; float64 copies rounded once from extended precision."""

    params: dict
    Q: np.ndarray          # d x d
    A: np.ndarray          # C x d
    M_D: np.ndarray        # C x d, Dirichlet map
    M_N: np.ndarray        # C x d, Neumann map
    residuals: dict = field(default_factory=dict)

    def M(self, bc: str) -> np.ndarray:
        """Map for a wall of type 'D' (Dirichlet) or 'N' (Neumann)."""
        return {"D": self.M_D, "N": self.M_N}[bc]


def gram_basis(d: int):
    """Householder QR of the matching-point Vandermonde matrix (step 1)."""
    xi = [mp.mpf(j - (d - 1)) for j in range(d)]
    V = mp.matrix(d, d)
    for j in range(d):
        for m in range(d):
            V[j, m] = xi[j] ** m
    Q, R = mp.qr(V)
    for m in range(d):                      # sign convention diag(R) > 0
        if R[m, m] < 0:
            for i in range(d):
                Q[i, m] = -Q[i, m]
                R[m, i] = -R[m, i]
    return V, Q, R


def gram_poly(Rinv, m: int, x):
    """P_m(x) = sum_k x^k (R^{-1})[k, m]."""
    d = Rinv.rows
    return mp.fsum((x ** k) * Rinv[k, m] for k in range(d))


def trig_row(x, K: int, T):
    row = [mp.mpf(1)]
    for k in range(1, K + 1):
        a = 2 * mp.pi * k * x / T
        row.append(mp.cos(a))
        row.append(mp.sin(a))
    return row


def build(params: dict | None = None) -> tuple[FCGramTables, dict]:
    """Build the tables (steps 1-5).  Returns (float64 tables, mp objects)."""
    p = dict(DEFAULT_PARAMS)
    if params:
        p.update(params)
    d, C, Z, E, n_os, K = p["d"], p["C"], p["Z"], p["E"], p["n_os"], p["K"]
    with mp.workdps(p["dps"]):
        T = mp.mpf(d + C + Z + E - 1)
        V, Q, R = gram_basis(d)
        Rinv = R ** -1
        match = [mp.mpf(-(d - 1)) + mp.mpf(i) / n_os for i in range((d - 1) * n_os + 1)]
        zero = [mp.mpf(C + 1) + mp.mpf(i) / n_os for i in range((Z - 1) * n_os + 1)]
        Amat = mp.matrix([trig_row(x, K, T) for x in match + zero])
        # exact least squares through the SVD pseudo-inverse (no truncation)
        U, S, Vt = mp.svd_r(Amat)
        nu = 2 * K + 1
        A = mp.matrix(C, d)
        res_match, res_zero = [], []
        coefs = []
        for m in range(d):
            rhs = [gram_poly(Rinv, m, x) for x in match] + [mp.mpf(0)] * len(zero)
            coef = [mp.mpf(0)] * nu
            for i in range(len(S)):
                ub = mp.fsum(U[r, i] * rhs[r] for r in range(len(rhs))) / S[i]
                for c in range(nu):
                    coef[c] += ub * Vt[i, c]
            coefs.append(coef)

            def g(x, coef=coef):
                return mp.fsum(a * b for a, b in zip(coef, trig_row(x, K, T)))

            res_match.append(max(abs(g(x) - gram_poly(Rinv, m, x)) for x in match))
            res_zero.append(max(abs(g(x)) for x in zero))
            for i in range(C):
                A[i, m] = g(mp.mpf(i + 1))
        M_D = A * Q.T
        # Neumann: derivative row delta_m = P_m'(0) = (R^{-1})[1, m]
        aug = mp.matrix(d + 1, d)
        for i in range(d):
            for m in range(d):
                aug[i, m] = Q[i, m]
        for m in range(d):
            aug[d, m] = Rinv[1, m]
        pinv = (aug.T * aug) ** -1 * aug.T       # full column rank: exact pinv
        G_N = mp.matrix(d, d)
        for i in range(d):
            for j in range(d):
                G_N[i, j] = pinv[i, j]
        M_N = A * G_N
        cond = S[0] / S[len(S) - 1]

        def f64(Mx):
            return np.array([[float(Mx[i, j]) for j in range(Mx.cols)] for i in range(Mx.rows)])

        tabs = FCGramTables(
            params=p, Q=f64(Q), A=f64(A), M_D=f64(M_D), M_N=f64(M_N),
            residuals=dict(match=[float(r) for r in res_match],
                           zero=[float(r) for r in res_zero],
                           cond=float(cond)))
        mpobj = dict(V=V, Q=Q, R=R, Rinv=Rinv, A=A, M_D=M_D, M_N=M_N, G_N=G_N,
                     coefs=coefs, T=T, match=match, zero=zero)
    return tabs, mpobj


# ---------------------------------------------------------------- table file
def _hex_rows(Mx: np.ndarray) -> list[str]:
    return [" ".join(float(v).hex() for v in row) for row in Mx]


def write_table(tabs: FCGramTables, path: str) -> None:
    p = tabs.params
    body = []
    for name in ("Q", "A", "M_D", "M_N"):
        Mx = getattr(tabs, name)
        body.append(f"{name} {Mx.shape[0]} {Mx.shape[1]}")
        body.extend(_hex_rows(Mx))
    digest = hashlib.sha256("\n".join(body).encode()).hexdigest()
    head = ["# FC(Gram) continuation tables (oracle construction: SVD pseudo-inverse)",
            "# params " + " ".join(f"{k}={p[k]}" for k in sorted(p)),
            "# residual_match " + " ".join(f"{r:.3e}" for r in tabs.residuals["match"]),
            "# residual_zero " + " ".join(f"{r:.3e}" for r in tabs.residuals["zero"]),
            f"# cond {tabs.residuals['cond']:.3e}",
            f"# sha256 {digest}"]
    with open(path, "w") as fh:
        fh.write("\n".join(head + body) + "\n")


def read_table(path: str) -> FCGramTables:
    mats, params, res = {}, {}, {"match": [], "zero": [], "cond": float("nan")}
    with open(path) as fh:
        lines = [ln.rstrip("\n") for ln in fh]
    i = 0
    while i < len(lines):
        ln = lines[i]
        if ln.startswith("# params"):
            for kv in ln.split()[2:]:
                k, v = kv.split("=")
                params[k] = int(v)
        elif ln.startswith("# residual_match"):
            res["match"] = [float(v) for v in ln.split()[2:]]
        elif ln.startswith("# residual_zero"):
            res["zero"] = [float(v) for v in ln.split()[2:]]
        elif ln.startswith("# cond"):
            res["cond"] = float(ln.split()[2])
        elif ln and not ln.startswith("#"):
            name, r, c = ln.split()
            r, c = int(r), int(c)
            rows = [[float.fromhex(v) for v in lines[i + 1 + k].split()] for k in range(r)]
            mats[name] = np.array(rows, dtype=np.float64).reshape(r, c)
            i += r
        i += 1
    return FCGramTables(params=params, Q=mats["Q"], A=mats["A"], M_D=mats["M_D"],
                        M_N=mats["M_N"], residuals=res)


def default_table_path(d: int = 5, C: int = 25) -> str:
    return os.path.join(TABLE_DIR, f"fcgram_d{d}_C{C}.txt")


def load(d: int = 5, C: int = 25) -> FCGramTables:
    """Committed oracle table (written by ``oracle/make_tables.py``)."""
    return read_table(default_table_path(d, C))
