"""A single pairwise contraction step (Section 5.4): C = sum over shared
indices of A * B, all index dimensions 2.

Labels list each operand's indices from the most significant address bit to
the least significant one (the last label has stride 1), i.e. numpy C order
of an array of shape (2,)*rank.  A label present in A and B but not in C is
summed; a label present in all three is a batch index.
"""
import string
import numpy as np


def _letters(labels_all):
    uniq = sorted(set(labels_all))
    pool = string.ascii_letters
    if len(uniq) > len(pool):
        raise ValueError("too many labels for einsum")
    return {lab: pool[i] for i, lab in enumerate(uniq)}


def einsum_step(a, b, la, lb, lc):
    """Reference contraction by numpy.einsum in complex128; flat result."""
    a = np.asarray(a, dtype=np.complex128).reshape((2,) * len(la))
    b = np.asarray(b, dtype=np.complex128).reshape((2,) * len(lb))
    m = _letters(list(la) + list(lb) + list(lc))
    spec = "".join(m[x] for x in la) + "," + "".join(m[x] for x in lb) + "->" + \
        "".join(m[x] for x in lc)
    return np.einsum(spec, a, b).reshape(-1)


def _decode(index, labels):
    """Bit values of each label for a linear index (last label = bit 0)."""
    r = len(labels)
    return {lab: (index >> (r - 1 - i)) & 1 for i, lab in enumerate(labels)}


def _encode(values, labels):
    idx = 0
    for lab in labels:
        idx = (idx << 1) | values[lab]
    return idx


def sampled_step(get_a, get_b, la, lb, lc, coords):
    """Entries of C at linear output indices ``coords`` by direct summation.

    ``get_a(idx)`` / ``get_b(idx)`` return complex entries of A / B at integer
    numpy arrays of linear indices (so A and B never need to be on the host
    in full).  For each output coordinate the 2^|K| products are formed and
    summed in complex128.
    """
    shared = [x for x in la if x in lb]
    summed = [x for x in shared if x not in lc]
    ks = len(summed)
    kvals = np.arange(1 << ks, dtype=np.int64)
    out = np.empty(len(coords), dtype=np.complex128)
    for n, c in enumerate(coords):
        fixed = _decode(int(c), lc)
        ia = np.zeros(1 << ks, dtype=np.int64)
        ib = np.zeros(1 << ks, dtype=np.int64)
        ra, rb = len(la), len(lb)
        for i, lab in enumerate(la):
            if lab in fixed:
                ia += fixed[lab] << (ra - 1 - i)
            else:
                j = summed.index(lab)
                ia += ((kvals >> j) & 1) << (ra - 1 - i)
        for i, lab in enumerate(lb):
            if lab in fixed:
                ib += fixed[lab] << (rb - 1 - i)
            else:
                j = summed.index(lab)
                ib += ((kvals >> j) & 1) << (rb - 1 - i)
        va = np.asarray(get_a(ia), dtype=np.complex128)
        vb = np.asarray(get_b(ib), dtype=np.complex128)
        out[n] = np.sum(va * vb)
    return out
