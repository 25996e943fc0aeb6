"""Reader for the text fixtures in this folder."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def flux_hand_cases():
    cases = []
    with open(os.path.join(HERE, "flux_hand_cases.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, qi, qj, n, F = [p.strip() for p in line.split("|")]
            cases.append((name, *(np.array([float(x) for x in s.split()]) for s in (qi, qj, n, F))))
    return cases


def unit_tet_dual():
    """{(a, b): 24 * area vector} of the unit tetrahedron's dual faces."""
    out = {}
    with open(os.path.join(HERE, "unit_tet_dual.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            ab, v = [p.strip() for p in line.split("|")]
            a, b = (int(x) for x in ab.split())
            out[(a, b)] = np.array([float(x) for x in v.split()])
    return out
