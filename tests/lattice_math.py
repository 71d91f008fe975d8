"""Implementation-independent lattice mathematics used to pin the oracle.

Everything here is integer enumeration or a closed form; nothing calls the oracle
or the HIP library.
"""
import itertools
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            out[k] = [int(t) for t in v] if len(v) > 1 else int(v[0])
    return out


def family_offsets(m: float):
    """Integer offsets o with 0 < |o|^2 <= m^2 (m = horizon in lattice spacings)."""
    r = int(np.floor(m)) + 1
    return np.array([o for o in itertools.product(range(-r, r + 1), repeat=3)
                     if 0 < o[0] ** 2 + o[1] ** 2 + o[2] ** 2 <= m * m], dtype=np.int64)


def slot_count(dims, m: float) -> int:
    """Directed slots of an L0 x L1 x L2 lattice: sum over offsets of prod (L_d - |o_d|)."""
    O = family_offsets(m)
    tot = 0
    for o in O:
        tot += int(np.prod([max(int(dims[d]) - abs(int(o[d])), 0) for d in range(3)]))
    return tot
