"""Brute-force state-vector simulation (the Schroedinger class of simulators
in Section 3.2; the state of n qubits needs 2^n amplitudes, Section 3.1).

Qubit 0 is the most significant bit of the state index, so the amplitude of
bitstring b is psi[sum_q b_q 2^(n-1-q)].

``projectors`` maps a canonical wire (q, s) to a bit value v: right after
the s-th two-qubit gate acting on qubit q, the projector |v><v| is applied
to q.  Summing over both values of v gives back the identity, so this
defines, independently of any tensor network, the contribution of one slice
(Section 5.1: slicing fixes a wire to each of its values and sums the
independent results).
"""
import numpy as np
from .gates import gate_matrix


def _apply_1q(psi, u, q):
    psi = np.tensordot(u, psi, axes=([1], [q]))
    return np.moveaxis(psi, 0, q)


def _apply_2q(psi, g, q0, q1):
    g4 = g.reshape(2, 2, 2, 2)
    psi = np.tensordot(g4, psi, axes=([2, 3], [q0, q1]))
    return np.moveaxis(psi, [0, 1], [q0, q1])


def statevector(circuit, projectors=None) -> np.ndarray:
    """Final state (2^n complex128) of ``circuit`` applied to |0...0>."""
    n = circuit.n_qubits
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    seg = [0] * n
    projectors = projectors or {}
    for g in circuit.gates:
        m = gate_matrix(g)
        if g.two_qubit:
            psi = _apply_2q(psi, m, g.q0, g.q1)
            for q in (g.q0, g.q1):
                seg[q] += 1
                v = projectors.get((q, seg[q]))
                if v is not None:
                    p = np.zeros((2, 2), dtype=np.complex128)
                    p[v, v] = 1.0
                    psi = _apply_1q(psi, p, q)
        else:
            psi = _apply_1q(psi, m, g.q0)
    return psi.reshape(-1)


def bit_index(bits) -> int:
    """State index of a full bitstring (qubit 0 = most significant bit)."""
    idx = 0
    for b in bits:
        idx = (idx << 1) | int(b)
    return idx


def amplitudes_sv(circuit, open_qubits, closed_bits, projectors=None) -> np.ndarray:
    """Amplitude batch from the state vector.

    Element j of the result has, for every i, the value of qubit
    ``open_qubits[i]`` equal to bit i of j (the first open qubit is the least
    significant bit of j).  ``closed_bits`` lists the bits of the remaining
    qubits in increasing qubit order.
    """
    n = circuit.n_qubits
    psi = statevector(circuit, projectors)
    open_qubits = list(open_qubits)
    closed = [q for q in range(n) if q not in open_qubits]
    if len(closed_bits) != len(closed):
        raise ValueError("closed_bits length mismatch")
    out = np.empty(1 << len(open_qubits), dtype=np.complex128)
    bits = [0] * n
    for q, b in zip(closed, closed_bits):
        bits[q] = int(b)
    for j in range(out.size):
        for i, q in enumerate(open_qubits):
            bits[q] = (j >> i) & 1
        out[j] = psi[bit_index(bits)]
    return out
