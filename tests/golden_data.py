"""Reader of the fixtures under tests/golden/ (values the paper states, each with the passage
that states it)."""
import os
from fractions import Fraction

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def paper_constants():
    """name -> float, or a list of floats for a value with several entries."""
    out = {}
    with open(os.path.join(GOLDEN, "paper_constants.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, rest = line.split("=", 1)
            value = rest.split(";", 1)[0].split()
            vals = [float(Fraction(v)) for v in value]
            out[name.strip()] = vals if len(vals) > 1 else vals[0]
    return out


def named_rows(fname):
    """name -> numpy array of the values of a `name v1 v2 ...` fixture (comments skipped)."""
    import numpy as np
    out = {}
    with open(os.path.join(GOLDEN, fname)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, *vals = line.split()
            out[name] = np.array([float(v) for v in vals])
    return out
