"""Loader for the paper-printed values in tests/golden/paper_tables.json."""
import json
import math
import os
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))


def tables():
    with open(os.path.join(HERE, "golden", "paper_tables.json")) as f:
        return json.load(f)


def exact(expr):
    """Evaluate an entry like '1/12', '(14-s7)/30' or '(-1+s7)/30' (s7 = sqrt 7)."""
    e = expr.replace(" ", "")
    if "s7" not in e:
        return float(Fraction(e))
    num, den = e.rsplit("/", 1)
    num = num.strip("()")
    a, sign = (num[:-3], num[-3]) if num.endswith(("+s7", "-s7")) else (None, None)
    if a is not None:
        return (float(Fraction(a)) + (1 if sign == "+" else -1) * math.sqrt(7)) / float(den)
    # forms like 14+s7 handled above; '-1+s7'
    raise ValueError(expr)
