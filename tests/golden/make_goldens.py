"""Write the stored oracle values of the GPU parity tests.

Calls only the CPU oracle (``oracle/``), the seeded input generators
(``rqcgen``) and the order helper of the tests (``tests/plan_order.py``,
index bookkeeping only).  The contraction orders and wire lists come from
the committed order fixtures next to this script (see export_orders.py):
they choose which sub-sums are formed and in which order, never a value.

    python tests/golden/make_goldens.py config2 [--jobs 4]
    python tests/golden/make_goldens.py share4 [--jobs 4]

config2: the 64 amplitudes of the 6x6 (1+14+1) circuit (seed 2), open
qubits 30..35, closed bits rqcgen.random_bits(30, 2): the sum of the 256
slices of order fixture a, cross-checked against the sum of the 1024
slices of order fixture b (another tree, other sliced wires).  Slicing
reaches the plain definition <b|U|0> exactly (Section 5.1), so the two
sums must agree to rounding.

share4: every slice of the 256-slice share of the 10x10 (1+20+1) circuit
(seed 4, all qubits closed, closed bits rqcgen.random_bits(100, 4)) of
order fixture share4_order: slice i fixes the enumerated sliced wires to
the bits of i and the share's fixed and single-valued wires to their
values.
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import rqcgen  # noqa: E402
from plan_order import oracle_order, oracle_wires_and_ids  # noqa: E402


def load_fixture(name):
    with open(os.path.join(HERE, name + ".json")) as f:
        return json.load(f)


def _circuit(fx):
    c = fx["circuit"]
    return rqcgen.grid_rqc(c["rows"], c["cols"], c["depth"], c["seed"])


def _work(args):
    name, bits, ids, threads = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(threads)
    except ImportError:
        pass
    fx = load_fixture(name)
    circ = _circuit(fx)
    groups, pairs = oracle_order(circ, fx["open"], fx)
    wires, oids = oracle_wires_and_ids(fx, ids)
    return oracle.slice_values_ordered(circ, fx["open"], bits, wires, oids, groups, pairs)


def slice_values(name, bits, ids, jobs):
    chunks = [list(ids[i::jobs]) for i in range(jobs)]
    threads = max(1, (os.cpu_count() or 1) // jobs)
    with ProcessPoolExecutor(jobs) as ex:
        parts = list(ex.map(_work, [(name, bits, c, threads) for c in chunks]))
    out = np.zeros((len(ids),) + parts[0].shape[1:], dtype=np.complex128)
    for i, part in enumerate(parts):
        out[i::jobs] = part
    return out


def write_rows(path, header, rows):
    with open(path, "w") as f:
        for line in header:
            f.write("# " + line + "\n")
        for idx, v in rows:
            f.write(f"{int(idx)} {float(v.real)!r} {float(v.imag)!r}\n")


def config2(jobs):
    bits = rqcgen.random_bits(30, 2)
    t = time.time()
    a = slice_values("config2_order_a", bits, list(range(256)), jobs).sum(axis=0)
    ta = time.time() - t
    t = time.time()
    b = slice_values("config2_order_b", bits, list(range(1024)), jobs).sum(axis=0)
    tb = time.time() - t
    n = 36
    agree = float(np.max(np.abs(a - b)) * 2 ** (n / 2))
    if agree > 1e-9:
        raise SystemExit(f"the two orders disagree: {agree}")
    pt = float(np.mean(np.abs(a) ** 2) * 2 ** n)
    header = [
        "Oracle amplitudes (complex128) of the 6x6-qubit (1+14+1) grid circuit,",
        "rqcgen.grid_rqc(6, 6, 14, 2); open qubits 30..35 (entry index bit i =",
        "qubit 30+i); closed bits rqcgen.random_bits(30, 2) for qubits 0..29.",
        "Sum of the 256 slices of config2_order_a.json (Section 5.1 slicing),",
        f"contracted by oracle.contract_ordered ({ta:.0f} s).  Cross-check: the 1024",
        "slices of config2_order_b.json (other tree, other wires) agree to",
        f"{agree:.2e} in units of 2^-18 ({tb:.0f} s).  Mean of 2^36 |a|^2 over the",
        f"batch: {pt:.3f} (Porter-Thomas, Section 6.2: 1 in expectation).",
        "Written by tests/golden/make_goldens.py config2.",
        "columns: entry re im",
    ]
    write_rows(os.path.join(HERE, "config2_amplitudes.txt"), header, enumerate(a))
    print("config2:", agree, pt)


def batch6(jobs):
    """64 entries of the 2^21-amplitude batch of the 6x6 (1+12+1) circuit
    rqcgen.grid_rqc(6, 6, 12, 2) with qubits 15..35 open and qubits 0..14 at
    rqcgen.random_bits(15, 3): the entries whose qubits 15..29 equal
    rqcgen.random_bits(15, 4), i.e. the amplitudes with those 30 qubits
    closed and qubits 30..35 open (entry j: bit i = qubit 30+i)."""
    bits = np.concatenate([rqcgen.random_bits(15, 3), rqcgen.random_bits(15, 4)])
    t = time.time()
    a = slice_values("batch6_order", bits, list(range(64)), jobs).sum(axis=0)
    dt = time.time() - t
    header = [
        "Oracle amplitudes (complex128) of the 6x6-qubit (1+12+1) grid circuit",
        "rqcgen.grid_rqc(6, 6, 12, 2) with qubits 0..14 closed at",
        "rqcgen.random_bits(15, 3), qubits 15..29 closed at rqcgen.random_bits(15, 4)",
        "and qubits 30..35 open (entry j: bit i = qubit 30+i): 64 entries of the",
        "2^21-amplitude correlated batch with qubits 15..35 open (Appendix A).",
        f"Sum of the 64 slices of batch6_order.json ({dt:.0f} s).",
        "Written by tests/golden/make_goldens.py batch6.",
        "columns: entry re im",
    ]
    write_rows(os.path.join(HERE, "batch6_amplitudes.txt"), header, enumerate(a))
    print("batch6: mean 2^36|a|^2", float(np.mean(np.abs(a) ** 2) * 2 ** 36))


def share4(jobs):
    bits = rqcgen.random_bits(100, 4)
    fx = load_fixture("share4_order")
    t = time.time()
    vals = slice_values("share4_order", bits, list(range(256)), jobs)[:, 0]
    dt = time.time() - t
    n_total = len(fx["sliced_wires"]) + len(fx["fixed_wires"])
    header = [
        "Oracle slice values (complex128) of the 256-slice share of the 10x10-qubit",
        "(1+20+1) grid circuit rqcgen.grid_rqc(10, 10, 20, 4), all qubits closed,",
        "bits rqcgen.random_bits(100, 4).  Slice i: the enumerated sliced wires of",
        "share4_order.json at the bits of i, its fixed and single-valued wires at",
        f"their values ({n_total} sliced wires in all; Section 5.1).  Contracted by",
        f"oracle.contract_ordered along the fixture's tree ({dt:.0f} s).",
        "Written by tests/golden/make_goldens.py share4.",
        "columns: slice re im",
    ]
    write_rows(os.path.join(HERE, "share4_slices.txt"), header, enumerate(vals))
    print("share4: max |s|", float(np.max(np.abs(vals))), "natural",
          oracle.natural_slice_scale(100, n_total))


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["config2", "share4", "batch6"])
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    {"config2": config2, "share4": share4, "batch6": batch6}[a.which](a.jobs)
