"""Build the FC(Gram) continuation matrices used by the library (offline).

The FC(Gram) variant (closing paragraph of the paper's FC section) applies
precomputed matrices to the d wall-adjacent values of every line; the
construction is fixed by these choices:

* matching points xi_j = j - (d-1) (grid units, wall at xi = 0);
* Gram basis: orthonormalise 1, xi, .., xi^{d-1} over the matching points
  (classical Gram-Schmidt at high precision, positive leading coefficients);
* blend-to-zero continuation g_m of each Gram polynomial: the least-squares
  trigonometric polynomial of period T = d + C + Z + E - 1 with K harmonics
  that equals the polynomial on [-(d-1), 0] and 0 on [C+1, C+Z], both sampled
  every 1/n_os (solved here by Householder QR);
* Dirichlet map M_D[i-1, :] = sum_m g_m(i) q_m^T, i = 1..C;
* Neumann map: the least-squares coefficients with one appended derivative
  row (value 0) as in the paper's Neumann treatment, M_N = A G_N.

Output: ``fcgram_d5_C25.txt`` next to this script, one matrix entry per line
as a C99 hex float.  Run:  python paper_2606_06247_amd/tables/make_fcgram.py
"""
from __future__ import annotations

import os

import mpmath as mp

PARAMS = dict(d=5, C=25, Z=12, E=25, n_os=20, K=25, dps=64)
HERE = os.path.dirname(os.path.abspath(__file__))


def gram_schmidt(d):
    """Orthonormal polynomial coefficient vectors (monomial basis) over the
    matching points; returns (coeffs[m][k], values[m][j])."""
    pts = [mp.mpf(j - (d - 1)) for j in range(d)]
    polys, vals = [], []
    for m in range(d):
        c = [mp.mpf(0)] * d
        c[m] = mp.mpf(1)
        for _ in range(2):                       # re-orthogonalise once
            v = [mp.fsum(c[k] * x ** k for k in range(d)) for x in pts]
            for pc, pv in zip(polys, vals):
                dot = mp.fsum(a * b for a, b in zip(v, pv))
                c = [a - dot * b for a, b in zip(c, pc)]
        v = [mp.fsum(c[k] * x ** k for k in range(d)) for x in pts]
        nrm = mp.sqrt(mp.fsum(a * a for a in v))
        c = [a / nrm for a in c]
        polys.append(c)
        vals.append([a / nrm for a in v])
    return polys, vals


def build():
    p = PARAMS
    d, C, Z, E, n_os, K = p["d"], p["C"], p["Z"], p["E"], p["n_os"], p["K"]
    mp.mp.dps = p["dps"]
    T = mp.mpf(d + C + Z + E - 1)
    polys, vals = gram_schmidt(d)

    def poly(m, x):
        return mp.fsum(polys[m][k] * x ** k for k in range(d))

    def basis(x):
        out = [mp.mpf(1)]
        for k in range(1, K + 1):
            out += [mp.cos(2 * mp.pi * k * x / T), mp.sin(2 * mp.pi * k * x / T)]
        return out

    xs_m = [-(d - 1) + mp.mpf(i) / n_os for i in range((d - 1) * n_os + 1)]
    xs_z = [C + 1 + mp.mpf(i) / n_os for i in range((Z - 1) * n_os + 1)]
    B = mp.matrix([basis(x) for x in xs_m + xs_z])
    A = [[mp.mpf(0)] * d for _ in range(C)]
    for m in range(d):
        rhs = mp.matrix([poly(m, x) for x in xs_m] + [0] * len(xs_z))
        coef, _ = mp.qr_solve(B, rhs)
        for i in range(C):
            A[i][m] = mp.fsum(a * b for a, b in zip(coef, basis(mp.mpf(i + 1))))
    # Q[j][m] = value of Gram polynomial m at matching point j
    Q = [[vals[m][j] for m in range(d)] for j in range(d)]
    MD = [[mp.fsum(A[i][m] * Q[j][m] for m in range(d)) for j in range(d)] for i in range(C)]
    # Neumann: least squares of [Q; delta^T] c = [f; 0] for each unit f
    delta = [polys[m][1] for m in range(d)]          # P_m'(0) = coefficient of xi
    aug = mp.matrix(d + 1, d)
    for j in range(d):
        for m in range(d):
            aug[j, m] = Q[j][m]
    for m in range(d):
        aug[d, m] = delta[m]
    GN = [[mp.mpf(0)] * d for _ in range(d)]
    for j in range(d):
        rhs = mp.matrix(d + 1, 1)
        rhs[j] = 1
        c, _ = mp.qr_solve(aug, rhs)
        for m in range(d):
            GN[m][j] = c[m]
    MN = [[mp.fsum(A[i][m] * GN[m][j] for m in range(d)) for j in range(d)] for i in range(C)]
    return MD, MN


def main():
    MD, MN = build()
    p = PARAMS
    path = os.path.join(HERE, f"fcgram_d{p['d']}_C{p['C']}.txt")
    with open(path, "w") as fh:
        fh.write("# FC(Gram) maps for the library; params "
                 + " ".join(f"{k}={v}" for k, v in sorted(p.items())) + "\n")
        for name, M in (("dirichlet", MD), ("neumann", MN)):
            fh.write(f"{name} {len(M)} {len(M[0])}\n")
            for row in M:
                for v in row:
                    fh.write(float(v).hex() + "\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
