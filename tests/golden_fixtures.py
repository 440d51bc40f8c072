"""Readers for the closed-form fixtures under tests/golden/ (each file states its derivation)."""
import os
from fractions import Fraction
from math import sqrt

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _eval(expr):
    return float(eval(expr, {"__builtins__": {}}, {"sqrt": sqrt, "Fraction": Fraction}))


def read_table(name):
    """{(kind, key): [values]} from a fixture file; comment lines start with '#'."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            out[(parts[0], int(parts[1]))] = [_eval(e) for e in parts[2:]]
    return out
