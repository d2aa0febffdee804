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
