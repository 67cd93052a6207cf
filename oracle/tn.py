"""Tensor-network amplitudes (Section 3.2, tensor approach; Section 5.1 slicing).

Network: one tensor per gate -- a single-qubit gate is the rank-2 tensor
U[out, in], a two-qubit gate the rank-4 tensor G[out0, out1, in0, in1] --
plus the vector |0> on every input wire and, on every closed output qubit q,
the vector e_{b_q}.  Open output qubits keep their last wire as a free
index.  Contracting all tensors gives <b|U|0...0> for every value of the
open qubits.

Canonical wires: the wire (q, s), s >= 1, is the output index of the s-th
two-qubit gate acting on qubit q (the wire segment that leaves that gate,
before any following single-qubit gate).  Slicing fixes such a wire to a
value v in every tensor that carries it; the contraction then gives one
slice, and the sum over all 2^S values of the S sliced wires gives the full
amplitude (Section 5.1).  The bit j of a slice id is the value of the j-th
sliced wire.

Contraction order: plain greedy -- repeatedly contract the pair of tensors
sharing an index that minimises size(C) - size(A) - size(B), ties broken by
the smaller (id A, id B).  The order only changes rounding, never the value.
"""
import heapq
import itertools
import numpy as np
from .gates import gate_matrix


class _Net:
    def __init__(self):
        self.tensors = {}      # id -> (array, labels list)
        self.next_id = 0
        self.next_label = 0

    def label(self):
        self.next_label += 1
        return self.next_label - 1

    def add(self, arr, labels):
        assert arr.ndim == len(labels)
        self.tensors[self.next_id] = (np.asarray(arr, dtype=np.complex128), list(labels))
        self.next_id += 1


def wire_labels(circuit):
    """Map canonical wire (q, s) -> its label in ``build_network`` (s >= 1)."""
    net, wires, _ = _build(circuit, None, None)
    return wires


def _build(circuit, open_qubits, closed_bits):
    n = circuit.n_qubits
    net = _Net()
    cur = [0] * n
    seg = [0] * n
    wires = {}
    zero = np.array([1.0, 0.0], dtype=np.complex128)
    for q in range(n):
        lab = net.label()
        net.add(zero, [lab])
        cur[q] = lab
    for g in circuit.gates:
        m = gate_matrix(g)
        if g.two_qubit:
            la, lb = net.label(), net.label()
            net.add(m.reshape(2, 2, 2, 2), [la, lb, cur[g.q0], cur[g.q1]])
            cur[g.q0], cur[g.q1] = la, lb
            for q, lab in ((g.q0, la), (g.q1, lb)):
                seg[q] += 1
                wires[(q, seg[q])] = lab
        else:
            lab = net.label()
            net.add(m, [lab, cur[g.q0]])
            cur[g.q0] = lab
    out_labels = None
    if open_qubits is not None:
        open_qubits = list(open_qubits)
        closed = [q for q in range(n) if q not in open_qubits]
        if len(closed_bits) != len(closed):
            raise ValueError("closed_bits length mismatch")
        for q, b in zip(closed, closed_bits):
            e = np.zeros(2, dtype=np.complex128)
            e[int(b)] = 1.0
            net.add(e, [cur[q]])
        out_labels = [cur[q] for q in open_qubits]
    return net, wires, out_labels


def build_network(circuit, open_qubits, closed_bits, sliced=None, slice_id=0):
    """Tensors (list of (array, labels)) and the open output labels.

    ``sliced`` is a list of canonical wires (q, s); bit j of ``slice_id`` is
    the value given to ``sliced[j]``.
    """
    net, wires, out_labels = _build(circuit, open_qubits, closed_bits)
    fixed = {}
    for j, w in enumerate(sliced or []):
        if w not in wires:
            raise ValueError(f"wire {w} does not exist")
        fixed[wires[w]] = (slice_id >> j) & 1
    tensors = []
    for tid in sorted(net.tensors):
        arr, labs = net.tensors[tid]
        for lab, v in fixed.items():
            if lab in labs:
                ax = labs.index(lab)
                arr = np.take(arr, v, axis=ax)
                labs = labs[:ax] + labs[ax + 1:]
        tensors.append((arr, labs))
    return tensors, out_labels


def _size(labels):
    return 1 << len(labels)


def contract_network(tensors, out_labels):
    """Contract all tensors greedily; return the array over ``out_labels``
    flattened so that ``out_labels[0]`` is the least significant bit."""
    live = {i: (a, list(l)) for i, (a, l) in enumerate(tensors)}
    owners = {}
    for i, (_, labs) in live.items():
        for lab in labs:
            owners.setdefault(lab, set()).add(i)
    keep_always = set(out_labels)
    next_id = len(tensors)

    def result_labels(la, lb, ia, ib):
        out = []
        for lab in la + lb:
            if lab in out:
                continue
            others = owners.get(lab, set()) - {ia, ib}
            if lab in keep_always or others or not (lab in la and lab in lb):
                out.append(lab)
        return out

    heap = []

    def push_pairs(i):
        _, la = live[i]
        seen = set()
        for lab in la:
            for j in owners.get(lab, ()):
                if j == i or j in seen:
                    continue
                seen.add(j)
                a, b = (i, j) if i < j else (j, i)
                lc = result_labels(live[a][1], live[b][1], a, b)
                cost = _size(lc) - _size(live[a][1]) - _size(live[b][1])
                heapq.heappush(heap, (cost, a, b))

    for i in sorted(live):
        push_pairs(i)

    while heap:
        cost, a, b = heapq.heappop(heap)
        if a not in live or b not in live:
            continue
        (ta, la), (tb, lb) = live[a], live[b]
        lc_now = result_labels(la, lb, a, b)
        if _size(lc_now) - _size(la) - _size(lb) != cost:
            heapq.heappush(heap, (_size(lc_now) - _size(la) - _size(lb), a, b))
            continue
        shared = [lab for lab in la if lab in lb]
        summed = [lab for lab in shared if lab not in lc_now]
        batch = [lab for lab in shared if lab in lc_now]
        if batch:
            raise NotImplementedError("an index shared by three tensors")
        tc = np.tensordot(ta, tb, axes=([la.index(x) for x in summed],
                                         [lb.index(x) for x in summed]))
        lc = [x for x in la if x not in summed] + [x for x in lb if x not in summed]
        del live[a], live[b]
        for lab in la:
            owners[lab].discard(a)
        for lab in lb:
            owners[lab].discard(b)
        c = next_id
        next_id += 1
        live[c] = (tc, lc)
        for lab in lc:
            owners.setdefault(lab, set()).add(c)
        push_pairs(c)

    # Disconnected pieces (scalars or open wires): outer products in id order.
    ids = sorted(live)
    res, rl = live[ids[0]]
    for i in ids[1:]:
        t, l = live[i]
        res = np.tensordot(res, t, axes=0)
        rl = rl + l
    if sorted(rl) != sorted(out_labels):
        raise RuntimeError("contraction left unexpected labels")
    order = [rl.index(lab) for lab in reversed(out_labels)]
    return np.transpose(res, order).reshape(-1) if order else np.asarray(res).reshape(1)


def contract_ordered(tensors, out_labels, groups, pairs):
    """Contract along an order given as data (the order changes rounding and
    cost, never the value).

    ``groups`` partitions the tensor indices; each group is first contracted
    in its listed order and becomes node ``g``.  ``pairs`` then lists
    contractions (a, b) of live nodes; the i-th pair creates node
    ``len(groups) + i``.  A label shared by the two operands is summed when
    no other live tensor carries it and it is not an output label.  Returns
    the array over ``out_labels`` flattened as in ``contract_network``.
    """
    seen = sorted(i for g in groups for i in g)
    if seen != list(range(len(tensors))):
        raise ValueError("groups must partition the tensors")
    live = {}
    owners = {}
    keep = set(out_labels)

    def add(nid, arr, labs):
        live[nid] = (arr, labs)
        for lab in labs:
            owners.setdefault(lab, set()).add(nid)

    def drop(nid):
        arr, labs = live.pop(nid)
        for lab in labs:
            owners[lab].discard(nid)
        return arr, labs

    def merge(x, y, nid):
        ta, la = drop(x)
        tb, lb = drop(y)
        summed = [lab for lab in la if lab in lb and lab not in keep and not owners.get(lab)]
        shared = [lab for lab in la if lab in lb]
        if len(shared) != len(summed):
            raise NotImplementedError("an index shared by three tensors")
        tc = np.tensordot(ta, tb, axes=([la.index(x) for x in summed], [lb.index(x) for x in summed]))
        add(nid, tc, [x for x in la if x not in summed] + [x for x in lb if x not in summed])

    # Tensors are registered under temporary ids first so that the summation
    # rule sees every tensor of the network.
    for i, (a, l) in enumerate(tensors):
        add(("t", i), np.asarray(a), list(l))
    for g, members in enumerate(groups):
        cur = ("t", members[0])
        for j, i in enumerate(members[1:]):
            nxt = ("g", g, j)
            merge(cur, ("t", i), nxt)
            cur = nxt
        arr, labs = drop(cur)
        add(g, arr, labs)
    for i, (a, b) in enumerate(pairs):
        merge(a, b, len(groups) + i)
    ids = sorted(live, key=str)
    res, rl = live[ids[0]]
    for i in ids[1:]:
        t, l = live[i]
        res = np.tensordot(res, t, axes=0)
        rl = rl + l
    if sorted(rl) != sorted(out_labels):
        raise RuntimeError("contraction left unexpected labels")
    order = [rl.index(lab) for lab in reversed(out_labels)]
    return np.transpose(res, order).reshape(-1) if order else np.asarray(res).reshape(1)


def slice_values_ordered(circuit, open_qubits, closed_bits, sliced, slice_ids, groups, pairs):
    """``slice_values_tn`` with the contraction order given as data."""
    res = []
    for sid in slice_ids:
        tensors, out = build_network(circuit, open_qubits, closed_bits, sliced, int(sid))
        res.append(contract_ordered(tensors, out, groups, pairs))
    return np.array(res)


def amplitudes_tn(circuit, open_qubits, closed_bits):
    """Amplitude batch by unsliced contraction (batch order as in the state
    vector oracle: open_qubits[0] is the least significant bit)."""
    tensors, out = build_network(circuit, open_qubits, closed_bits)
    return contract_network(tensors, out)


def slice_values_tn(circuit, open_qubits, closed_bits, sliced, slice_ids):
    """Per-slice amplitude batches: array (len(slice_ids), 2^n_open)."""
    res = []
    for sid in slice_ids:
        tensors, out = build_network(circuit, open_qubits, closed_bits, sliced, int(sid))
        res.append(contract_network(tensors, out))
    return np.array(res)


def all_slice_ids(n_sliced):
    return list(range(1 << n_sliced))


def iter_assignments(n):
    return itertools.product((0, 1), repeat=n)
