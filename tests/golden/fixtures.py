"""Readers for the small text fixtures in this folder (values printed in the paper)."""
import os
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))


def _lines(name):
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


def weno7_linear_coefficients():
    """{offset: Fraction} of eq:f7."""
    return {int(o): Fraction(int(n), int(d)) for o, n, d in _lines("weno7_linear_reconstruction.txt")}


def key_values(name):
    return {k: float(v) for k, v in _lines(name)}
