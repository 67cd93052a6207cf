"""Turn a plan's exported contraction tree into an order for the oracle's
own tensors (``oracle.contract_ordered``), so that the oracle can check
slices of networks whose plain greedy order would not fit in memory.

The order is data: it changes the oracle's cost and rounding, never the
value it computes.  The grouping follows the canonical wires of Section 3.2:
a qubit's |0> input and the single-qubit gates before its first two-qubit
gate join that gate; single-qubit gates between two two-qubit gates join the
later one; the trailing gates and the output projector join the last one.
"""


def oracle_order(circuit, open_qubits, export):
    n = circuit.n_qubits
    gates = circuit.gates
    n_t = n + len(gates)
    open_set = set(open_qubits)
    closed = [q for q in range(n) if q not in open_set]
    cap_index = {q: n_t + i for i, q in enumerate(closed)}
    two_q = [gi for gi, g in enumerate(gates) if g.two_qubit]
    group_of_gate = {gi: j for j, gi in enumerate(two_q)}
    groups = [[n + gi] for gi in two_q]
    pending = {q: [q] for q in range(n)}
    last = {}
    for gi, g in enumerate(gates):
        if g.two_qubit:
            j = group_of_gate[gi]
            for q in (g.q0, g.q1):
                groups[j].extend(pending[q])
                pending[q] = []
                last[q] = j
        else:
            pending[g.q0].append(n + gi)
    for q in range(n):
        if q not in last:
            raise ValueError(f"qubit {q} has no two-qubit gate")
        groups[last[q]].extend(pending[q])
        if q in cap_index:
            groups[last[q]].append(cap_index[q])
    # Plan leaf i is the i-th two-qubit gate: check that it touches the same
    # two qubits.
    labels = export["labels"]
    leaves = export["leaves"]
    if len(leaves) != len(two_q):
        raise ValueError("plan leaves do not match the two-qubit gates")
    for j, gi in enumerate(two_q):
        qs = {labels[x][1] for x in leaves[j]}
        if not qs <= {gates[gi].q0, gates[gi].q1}:
            raise ValueError(f"plan leaf {j} does not match gate {gi}")
    node = {i: i for i in range(len(leaves))}
    pairs = []
    for i, st in enumerate(export["steps"]):
        pairs.append((node[st["a"]], node[st["b"]]))
        node[st["node"]] = len(groups) + i
    return groups, pairs


def oracle_wires_and_ids(export, local_ids):
    """The wires the oracle fixes for a plan's slices and the matching slice
    ids: the enumerated sliced wires (bits of the local id), then the share's
    fixed wires and the pruned single-valued wires at their values.  Fixing
    a pruned wire drops only zero terms (pinned on the CPU), and keeps the
    oracle's intermediates along the plan's order as narrow as the plan's."""
    loc = [tuple(w) for w in export["sliced_wires"]]
    rest = [w for w in export["fixed_wires"]] + [w for w in export["pruned_wires"]]
    wires = loc + [tuple(w[:2]) for w in rest]
    high = 0
    for i, w in enumerate(rest):
        high |= int(w[2]) << i
    return wires, [int(s) | (high << len(loc)) for s in local_ids]
