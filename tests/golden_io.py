"""Reader for the text fixtures under tests/golden (values printed in the paper)."""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def num(tok: str) -> float:
    return float(Fraction(tok))


def lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                yield ln.split()


def read_matrix(rows_iter, k):
    return np.array([[num(t) for t in next(rows_iter)] for _ in range(k)])
