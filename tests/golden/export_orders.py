"""Write the contraction-order fixtures that the stored oracle values are
computed along (run once; the output is committed next to this script).

A fixture holds the sliced wires of a plan, the wires its planner fixed (a
slice share) or found single-valued, and its contraction tree.  These are
data for the oracle: they choose which sub-sums are formed and in which
order pairs of tensors are contracted (Section 5.1: slices are independent
sub-tasks whose sum is the amplitude; the order changes rounding, never the
value).  No value in a fixture comes from a device computation: the
planner runs on the host.

    python tests/golden/export_orders.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import rqcgen  # noqa: E402
import paper_2110_14502_amd as R  # noqa: E402

# name: (rows, cols, depth, circuit seed, open qubits, plan options)
FIXTURES = {
    # The 64-amplitude batch of the 6x6 (1+14+1) workload, 8 sliced wires.
    "config2_order_a": (6, 6, 14, 2, list(range(30, 36)),
                        dict(n_sliced=8, path_trials=1024, seed=42)),
    # The same batch along another tree and another set of sliced wires.
    "config2_order_b": (6, 6, 14, 2, list(range(30, 36)),
                        dict(n_sliced=10, path_trials=256, seed=7)),
    # 64 amplitudes of the 6x6 (1+12+1) circuit: a sub-batch of the 2^21-entry
    # correlated batch (qubits 15..35 open) with qubits 15..29 fixed.
    "batch6_order": (6, 6, 12, 2, list(range(30, 36)),
                     dict(n_sliced=6, path_trials=256, seed=3)),
    # A 256-slice share of the 10x10 (1+20+1) circuit, per-slice bound 2^24.
    "share4_order": (10, 10, 20, 4, [],
                     dict(max_log2_elems=24, path_trials=64, seed=4, n_local_sliced=8)),
}


def export(name):
    rows, cols, depth, cseed, openq, opts = FIXTURES[name]
    circ = rqcgen.grid_rqc(rows, cols, depth, cseed)
    plan = R.Plan(R.Network(R.Circuit.from_rqcgen(circ), openq), **opts)
    e = plan.export()
    return {
        "circuit": {"rows": rows, "cols": cols, "depth": depth, "seed": cseed},
        "open": openq,
        "plan_options": opts,
        "sliced_wires": e["sliced_wires"],
        "fixed_wires": e["fixed_wires"],
        "pruned_wires": e["pruned_wires"],
        "labels": e["labels"],
        "leaves": e["leaves"],
        "steps": [{"a": s["a"], "b": s["b"], "node": s["node"]} for s in e["steps"]],
    }


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(FIXTURES)):
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(export(name), f, separators=(",", ":"))
        print("wrote", name)
