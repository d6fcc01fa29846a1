"""Shared helpers of the GPU parity tests: build a library Problem and an oracle
Lattice from one spec, and compare results."""
from __future__ import annotations

import numpy as np

from oracle.lattice import Lattice


def spec(n, walled, vel=None, prs=None, dx=None, h=1.3):
    """n, walled in lattice order; vel / prs per axis ('D'|'N', 'D'|'N') or None."""
    nd = len(n)
    vel = tuple(vel) if vel else tuple(("D", "D") if w else None for w in walled)
    if prs is None:
        comp = {"D": "N", "N": "D"}
        prs = tuple((comp[v[0]], comp[v[1]]) if v else None for v in vel)
    if dx is None:
        wn = [k for k, w in zip(n, walled) if w]
        dx = 1.0 / (wn[0] - 1) if wn else 1.0 / n[0]
    return dict(n=tuple(n), walled=tuple(walled), vel=tuple(vel), prs=tuple(prs), dx=dx, h=h, nd=nd)


def lattice(s) -> Lattice:
    return Lattice(n=s["n"], walled=s["walled"], dx=s["dx"], vel_bc=s["vel"], prs_bc=s["prs"],
                   h_over_dx=s["h"])


def problem(s, precision="fp64", eig="spectral"):
    from paper_2606_06247_amd.api import Problem
    return Problem(n=s["n"], walled=s["walled"], dx=s["dx"], vel_bc=s["vel"], prs_bc=s["prs"],
                   h_over_dx=s["h"], precision=precision, eig=eig)


def rel_l2(got, ref) -> float:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)
