"""Reader for the small text fixtures in this folder (exact rationals)."""
from fractions import Fraction
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def _row(s):
    return [Fraction(x) for x in s.split()]


def load(name):
    out = {}
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, val = [x.strip() for x in line.split("=", 1)]
            rows = [_row(r) for r in val.split(";")]
            out[key] = rows if len(rows) > 1 else rows[0]
    return out
