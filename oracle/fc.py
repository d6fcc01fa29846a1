"""FC apply along walled axes (oracle side).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

Sec. "Fourier Continuation (FC) Algorithm", eq. eq:fc_extended: the extended
field equals f on the physical points and a continuation on the appended
points, and is periodic over the extended length.  Eq. eq:fc_2d applies the 1D
continuation along a walled axis on every line.

FC(Gram) form used here (continuation tables from ``oracle.fcgram``), for one
line f_0..f_{n-1} of a walled axis, extended to e_0..e_{n+C-1}:

    e[j]       = f[j]                                   j = 0..n-1
    e[n-1+i]   = (M_hi f_hi)[i] + (M_lo f_lo_rev)[C+1-i]  i = 1..C

with f_hi = (f_{n-d}, .., f_{n-1}) (high wall at index n-1) and
f_lo_rev = (f_{d-1}, .., f_0) (the low wall's data mirrored so that its wall
sits at the end of the matching interval); the low-wall continuation reaches
index n-1+i from the periodic image of index 0 at distance C+1-i.
M_hi / M_lo is the Dirichlet or Neumann map of that wall's boundary type.

With several walled axes the 1D map is applied along each walled axis to every
line of the current array, including the continuation lines created by an
earlier axis; the maps act on different indices, so the result does not depend
on the axis order (checked in tests).

Parity: pinned by P-FC1 (physical values copied unchanged), P-FC5/6/7
(smoothness and convergence) in ``tests/test_oracle_fc.py``.
"""
from __future__ import annotations

import numpy as np


def extend_line_axis(f: np.ndarray, axis: int, M_lo: np.ndarray, M_hi: np.ndarray) -> np.ndarray:
    """Extend ``f`` along numpy axis ``axis`` by C points (FC(Gram) apply)."""
    C, d = M_hi.shape
    g = np.moveaxis(np.asarray(f), axis, -1)
    n = g.shape[-1]
    if n < 2 * d:
        raise ValueError("walled axis needs at least 2d points")
    f_hi = g[..., n - d:]                  # f_{n-d} .. f_{n-1}
    f_lo_rev = g[..., d - 1::-1]           # f_{d-1} .. f_0
    cont_hi = f_hi @ M_hi.T                # [..., i-1] <-> continuation point i
    cont_lo = f_lo_rev @ M_lo.T            # [..., i-1] <-> distance i from the low wall
    cont = cont_hi + cont_lo[..., ::-1]    # point i gets low-wall row C+1-i
    e = np.concatenate([g, cont], axis=-1)
    return np.moveaxis(e, -1, axis)


def extend(f: np.ndarray, walled, bcs, tables, order=None) -> np.ndarray:
    """Extend along every walled axis.

    walled : per lattice axis (x, y[, z]) a bool
    bcs    : per lattice axis a pair ('D'|'N', 'D'|'N') for (low, high) walls
    tables : an object with ``M(bc)`` returning the C x d map
    order  : lattice-axis order in which to apply the 1D maps (default x, y, z)
    """
    ndim = f.ndim
    e = np.asarray(f, dtype=np.float64)
    axes = range(ndim) if order is None else order
    for a in axes:
        if walled[a]:
            lo, hi = bcs[a]
            e = extend_line_axis(e, ndim - 1 - a, tables.M(lo), tables.M(hi))
    return e


def restrict(e: np.ndarray, n) -> np.ndarray:
    """Physical part of an extended array; n is given in lattice order (x, y[, z])."""
    sl = tuple(slice(0, k) for k in reversed(tuple(n)))
    return e[sl]
