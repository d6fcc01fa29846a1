"""Loader of the library's FC(Gram) continuation maps (``tables/fcgram_d*_C*.txt``,
written by ``tables/make_fcgram.py``): one C99 hex float per line, row-major."""
from __future__ import annotations

import os

import numpy as np

_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tables")


def path(d: int = 5, C: int = 25) -> str:
    return os.path.join(_DIR, f"fcgram_d{d}_C{C}.txt")


def load(d: int = 5, C: int = 25) -> dict:
    with open(path(d, C)) as fh:
        lines = [ln.strip() for ln in fh if ln.strip() and not ln.startswith("#")]
    out, i = {}, 0
    while i < len(lines):
        name, r, c = lines[i].split()
        r, c = int(r), int(c)
        vals = [float.fromhex(v) for v in lines[i + 1:i + 1 + r * c]]
        out[name] = np.array(vals, dtype=np.float64).reshape(r, c)
        i += 1 + r * c
    if out["dirichlet"].shape != (C, d) or out["neumann"].shape != (C, d):
        raise ValueError("FC table has the wrong shape")
    return out
