"""Readers for the text fixtures under tests/golden (values printed in the paper)."""
import os
from fractions import Fraction

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


def fractions_table(name):
    """Map first token -> list of Fractions of the remaining numeric tokens."""
    out = {}
    for toks in _rows(name):
        vals = []
        for t in toks[1:]:
            try:
                vals.append(Fraction(t))
            except ValueError:
                continue
        out[toks[0]] = vals
    return out


def eq18():
    t = fractions_table("eq18_central_half_point.txt")
    return {k: [v[0] * c for c in v[1:]] for k, v in t.items()}


def eq11():
    t = fractions_table("eq11_correction.txt")
    return t["a2"][0], t["a4"][0]


def eq19():
    t = fractions_table("eq19_derivative.txt")
    return t["c1"][0], t["c2"][0], t["c3"][0]


def eq16():
    t = fractions_table("eq16_ideal_weights.txt")
    return t["gamma1"][0], t["gamma2"][0], t["gamma3"][0]


def eq17():
    return fractions_table("eq17_smoothness.txt")


def eq20():
    t = fractions_table("eq20_rk3.txt")
    return [t[s] for s in ("1", "2", "3")]
