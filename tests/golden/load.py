"""Readers for the small text fixtures in tests/golden/."""
import os
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))


def _lines(name):
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def hex_values(name):
    return [int(x, 16) for x in _lines(name)]


def keyed_fractions(name):
    """'key = a b ; c d' -> {key: [[Fraction]]} (rows separated by ';')."""
    out = {}
    for line in _lines(name):
        key, val = [s.strip() for s in line.split("=", 1)]
        rows = [[Fraction(t) for t in r.split()] for r in val.split(";")]
        out[key] = rows
    return out


def diffsolve_reference(name):
    """The differentiable-solve reference file: ({'X': max, ...}, {('X', r): (sum, abs sum)},
    {'X': [(i, j, value)], ...}), floats from their hex form."""
    maxabs, colsums, entries = {}, {}, {}
    for line in _lines(name):
        f = line.split()
        if f[0] == "maxabs":
            maxabs[f[1]] = float.fromhex(f[2])
        elif f[0] == "colsum":
            colsums[(f[1], int(f[2]))] = (float.fromhex(f[3]), float.fromhex(f[4]))
        elif f[0] == "entry":
            entries.setdefault(f[1], []).append((int(f[2]), int(f[3]), float.fromhex(f[4])))
    return maxabs, colsums, entries
