"""Spectral pressure-Poisson solve by dense per-axis transforms (oracle side).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

Sec. "Spatial discretisation of pressure": the PPE is solved by a transform
that diagonalises the Laplacian, DCT-I for collocated Neumann walls
(eq. DCTI4PPE, read as the tensor product of 1D DCT-I transforms) and a DFT on
periodic axes (eq. DCTDFT_PPE); in transform space the solve is a division by
the sum of the per-axis eigenvalues (eq. division4PPE).  Readings:
* Dirichlet pressure walls (phi = 0) use DST-I; one Dirichlet and one Neumann
  wall use the quarter-wave sine / cosine bases (the transform types of the
  FFT-based Poisson solvers the paper points to);
* eigenvalues: SPECTRAL (exact wavenumbers of the basis, the default, since
  the solver is called spectral), FD2 (second-order finite differences), or
  SPH (sum of squared gradient-symbol magnitudes, all-periodic lattices only);
* phi_hat = -b_hat / sum_a mu_a;  a mode whose eigenvalue sum vanishes (the
  constant mode of an all-Neumann / periodic lattice) gets phi_hat = 0.

Per axis of n physical points with spacing dx (N' = n - 1):

  type  unknowns j      basis (mode l)                   mu_SPECTRAL
  P     0..n-1          exp(2 pi i k j / n)              (2 pi k~ / (n dx))^2, k~ signed, Nyquist +n/2
  NN    0..n-1          cos(pi l j / N'),  l=0..n-1      (pi l / (N' dx))^2
  DD    1..n-2          sin(pi l j / N'),  l=1..n-2      (pi l / (N' dx))^2
  DN    1..n-1          sin(pi (2l+1) j / (2N')), l=0..n-2   ((l+1/2) pi / (N' dx))^2
  ND    0..n-2          cos(pi (2l+1) j / (2N')), l=0..n-2   as DN

The oracle builds each synthesis matrix from these definitions, inverts it
(numpy.linalg.inv, a library primitive) for the analysis, and applies both by
tensor contraction along each axis.  No FFT is used.

Parity: pinned by exact recovery of manufactured basis sums (P-PPE1), by
scipy.sparse.linalg.spsolve on the assembled 3/5/7-point operator for the FD2
family (P-PPE2), the zero-mode convention (P-PPE3) and single-mode eigen tests
(P-PPE4) in ``tests/test_oracle_ppe.py``.
"""
from __future__ import annotations

import numpy as np


def axis_kind(lat, a: int) -> str:
    if not lat.walled[a]:
        return "P"
    lo, hi = lat.prs_bc[a]
    return lo + hi                       # 'NN', 'DD', 'DN', 'ND'


def axis_basis(kind: str, n: int, dx: float, family: str = "spectral"):
    """(unknown indices, synthesis matrix S[j, l], eigenvalues mu[l])."""
    Np = n - 1
    if kind == "P":
        j = np.arange(n)
        k = np.arange(n)
        S = np.exp(2j * np.pi * np.outer(j, k) / n)
        ks = np.where(k <= n // 2, k, k - n).astype(np.float64)
        if family == "spectral":
            mu = (2 * np.pi * ks / (n * dx)) ** 2
        else:
            mu = 4.0 / dx ** 2 * np.sin(np.pi * k / n) ** 2
        return j, S, mu
    if kind == "NN":
        j = np.arange(n)
        l = np.arange(n)
        S = np.cos(np.pi * np.outer(j, l) / Np)
        th = np.pi * l / Np
    elif kind == "DD":
        j = np.arange(1, n - 1)
        l = np.arange(1, n - 1)
        S = np.sin(np.pi * np.outer(j, l) / Np)
        th = np.pi * l / Np
    elif kind == "DN":
        j = np.arange(1, n)
        l = np.arange(0, n - 1)
        S = np.sin(np.pi * np.outer(j, 2 * l + 1) / (2 * Np))
        th = np.pi * (2 * l + 1) / (2 * Np)
    elif kind == "ND":
        j = np.arange(0, n - 1)
        l = np.arange(0, n - 1)
        S = np.cos(np.pi * np.outer(j, 2 * l + 1) / (2 * Np))
        th = np.pi * (2 * l + 1) / (2 * Np)
    else:
        raise ValueError(kind)
    if family == "spectral":
        mu = (th / dx) ** 2
    else:
        mu = 4.0 / dx ** 2 * np.sin(th / 2.0) ** 2
    return j, S, mu


def _apply_axis(x, M, npax):
    """Contract matrix M (rows = output index) with array x along numpy axis npax."""
    x = np.moveaxis(x, npax, -1)
    y = x @ M.T
    return np.moveaxis(y, -1, npax)


def sph_eigenvalues(lat):
    """mu_SPH(k) = sum_a sigma_a(k)^2, S_a = i sigma_a = DFT of the gradient taps
    on the physical periodic lattice (all axes periodic)."""
    from . import kernels, operators
    if any(lat.walled):
        raise ValueError("SPH eigenvalues need an all-periodic lattice")
    tl = kernels.taps(lat.ndim, lat.dx, lat.h_over_dx)
    mu = np.zeros(lat.shape)
    for a in range(lat.ndim):
        ker = operators.corner_wrapped_kernel(lat.shape, [(s, float(g[a])) for s, g, _ in tl])
        Sa = np.fft.fftn(ker)
        mu += (Sa.imag) ** 2
    return mu


def solve(b: np.ndarray, lat, family: str = "spectral", return_diag: bool = False):
    """phi with lap(phi) = b under the lattice's pressure wall types."""
    b = np.asarray(b, dtype=np.float64)
    nd = lat.ndim
    idx, Ss, mus, kinds = [], [], [], []
    for a in range(nd):
        kind = axis_kind(lat, a)
        fam = "spectral" if family == "sph" else family
        j, S, mu = axis_basis(kind, lat.n[a], lat.dx, fam)
        idx.append(j)
        Ss.append(S)
        mus.append(mu)
        kinds.append(kind)
    # restrict b to the unknowns
    sl = np.ix_(*[idx[nd - 1 - ax] for ax in range(nd)])
    x = b[sl].astype(np.complex128)
    # analysis
    for a in range(nd):
        x = _apply_axis(x, np.linalg.inv(Ss[a]), nd - 1 - a)
    # eigenvalue sum on the mode grid (numpy order)
    if family == "sph":
        musum = sph_eigenvalues(lat)
    else:
        musum = np.zeros(x.shape)
        for a in range(nd):
            shp = [1] * nd
            shp[nd - 1 - a] = -1
            musum = musum + mus[a].reshape(shp)
    bhat0 = x.flat[0]
    tol = 1e-14 * np.max(np.abs(musum))
    safe = np.where(np.abs(musum) > tol, musum, 1.0)
    phat = np.where(np.abs(musum) > tol, -x / safe, 0.0)
    # synthesis
    y = phat
    for a in range(nd):
        y = _apply_axis(y, Ss[a], nd - 1 - a)
    phi = np.zeros(lat.shape, dtype=np.float64)
    phi[sl] = y.real
    if return_diag:
        return phi, dict(bhat0=bhat0, kinds=kinds)
    return phi
