"""Readers for the text fixtures under tests/golden/ (values from the paper)."""
import os
import re

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _poly(tok):
    """Parse a polynomial in mu written as in the paper, e.g. 3\\mu^2+3\\mu."""
    tok = tok.replace("\\mu", "m")
    coef = [0.0, 0.0, 0.0]
    for sign, body in re.findall(r"([+-]?)([^+-]+)", tok):
        s = -1.0 if sign == "-" else 1.0
        mt = re.fullmatch(r"(\d*)(m(\^(\d))?)?", body)
        if mt is None:
            raise ValueError(tok)
        c = float(mt.group(1)) if mt.group(1) else 1.0
        p = 0 if mt.group(2) is None else (int(mt.group(4)) if mt.group(4) else 1)
        coef[p] += s * c
    return coef


def read_poly_matrix(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([_poly(t) for t in line.split()])
    return np.array(rows)  # shape (r, c, 3)


def eval_poly_matrix(P, mu):
    return P[..., 0] + P[..., 1] * mu + P[..., 2] * mu * mu


def read_matrix(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return np.array([[float(t) for t in l.split()] for l in f
                         if l.strip() and not l.startswith("#")])


def read_tables():
    out = {}
    with open(os.path.join(GOLDEN, "tables.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t, fam, n, col, val = line.split()
            out[(t, fam, int(n), col)] = float(val)
    return out
