"""Readers for the text fixtures in tests/golden (paper values, each file cites its source)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


def table1():
    out = {}
    for r in _rows("table1_components.txt"):
        out[r[0]] = {"pc": float(r[1]), "Tc": float(r[2]), "omega": float(r[3]),
                     "M": float(r[4]), "Rs": float(r[5])}
    return out


def _num(s):
    return np.nan if s == "-" else float(s)


def table2():
    keys = ["p", "Zl", "Zv", "x1", "y1", "r1l", "r2l", "r1v", "r2v", "gamma1"]
    return [dict(zip(keys, map(_num, r))) for r in _rows("table2_c3_nc5.txt")]


def maxwell():
    r = next(_rows("maxwell_pure_pr.txt"))
    return dict(zip(["a", "b", "omega", "T_over_Tc", "rho_l", "rho_v"], map(float, r)))
