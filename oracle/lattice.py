"""Lattice geometry for the oracle.

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

Readings (the paper's grid indexing in Sec. "Fourier Continuation (FC)
Algorithm" is inconsistent about whether y = 1 is a grid point):
* a walled axis has n points x_j = j dx, both walls are lattice points;
* a periodic axis has n points with the same isotropic spacing dx and period
  n dx;
* every axis is given in lattice order (x, y[, z]); numpy arrays are indexed
  [z][y][x] (x fastest), so lattice axis a is numpy axis ndim-1-a.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class Lattice:
    n: tuple                       # physical points per lattice axis (x, y[, z])
    walled: tuple                  # bool per lattice axis
    dx: float                      # isotropic spacing
    vel_bc: tuple = None           # per axis (low, high) in {'D', 'N'}; walled axes only
    prs_bc: tuple = None
    h_over_dx: float = 1.3
    C: int = 25
    d: int = 5
    kernel: str = "wendland_c2"    # or "g2", "g4", "g6", "g8", "g10" (Gaussian family)

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def shape(self) -> tuple:
        """numpy shape of a physical array."""
        return tuple(reversed(self.n))

    @property
    def ext(self) -> tuple:
        """extended points per lattice axis."""
        return tuple(k + (self.C if w else 0) for k, w in zip(self.n, self.walled))

    @property
    def ext_shape(self) -> tuple:
        return tuple(reversed(self.ext))


def complement(bc: str) -> str:
    """Pressure wall type paired with a velocity wall type: Dirichlet velocity
    goes with homogeneous Neumann pressure (eqs. BC_velocity, BC_pressure) and
    a Neumann velocity wall with a Dirichlet (phi = 0) pressure wall."""
    return {"D": "N", "N": "D"}[bc]


def walled_box(n: tuple, vel_bc=None, prs_bc=None, **kw) -> Lattice:
    """All axes walled, dx = 1/(n_0 - 1) (the unit box for square lattices)."""
    nd = len(n)
    vel = vel_bc or tuple(("D", "D") for _ in range(nd))
    prs = prs_bc or tuple((complement(a), complement(b)) for a, b in vel)
    return Lattice(n=tuple(n), walled=(True,) * nd, dx=1.0 / (n[0] - 1),
                   vel_bc=tuple(vel), prs_bc=tuple(prs), **kw)
