"""Reading the stored oracle values under tests/golden (written by
tests/golden/make_goldens.py, which calls only the oracle)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    """(indices, complex128 values) of tests/golden/<name>."""
    idx, val = [], []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            i, re_, im_ = line.split()
            idx.append(int(i))
            val.append(complex(float(re_), float(im_)))
    return np.array(idx), np.array(val, dtype=np.complex128)
