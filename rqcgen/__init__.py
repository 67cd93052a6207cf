"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the simulation method itself: it only
draws gate *names*, qubit indices, bitstrings and random tensor entries from
seeded numpy generators.  Gate matrices live separately in the oracle and in
the native library, each written from the definitions.

Workload shapes follow the paper's random quantum circuits: square grids of
qubits, depth written "(1+d+1)" (Section 3.1 and the performance-attributes
table), two-qubit fSim gates named in Section 5.2, and an "open" batch of
qubits whose amplitudes are produced together (Section 5.1, last paragraph).
The exact gate set and coupler pattern below are not fixed by the paper; the
reading used is:

* a leading layer of H on every qubit;
* ``d`` cycles, each a layer of random single-qubit gates drawn from
  {sqrt(X), sqrt(Y), sqrt(W)}, never repeating the previous draw on the same
  qubit, followed by fSim(pi/2, pi/6) on every coupler of class
  ``"ABCDCDAB"[cycle % 8]``;
* a trailing random single-qubit layer under the same no-repeat rule.

Coupler classes on an R x C grid with qubit (r, c) -> r*C + c: horizontal
(r,c)-(r,c+1) is A when c is even and B when c is odd; vertical (r,c)-(r+1,c)
is C when r is even and D when r is odd.
"""
from __future__ import annotations

from dataclasses import dataclass
import math
import numpy as np

# Gate kinds.  The integer codes equal the native library's rqc_gate_kind.
H, SQRT_X, SQRT_Y, SQRT_W, FSIM, U1, U2 = range(7)
KIND_NAMES = {H: "H", SQRT_X: "SQRT_X", SQRT_Y: "SQRT_Y", SQRT_W: "SQRT_W",
              FSIM: "FSIM", U1: "U1", U2: "U2"}
_ONE_QUBIT_DRAWS = (SQRT_X, SQRT_Y, SQRT_W)
PATTERN = "ABCDCDAB"

FSIM_THETA = math.pi / 2
FSIM_PHI = math.pi / 6


@dataclass(frozen=True)
class Gate:
    """One gate of a circuit: kind, qubits, fSim angles, optional matrix.

    ``q1`` is -1 for single-qubit gates.  ``u`` holds an explicit unitary for
    kinds U1 (2x2) and U2 (4x4) as a complex numpy array, row-major,
    ``u[out, in]`` with two-qubit basis index ``2*b(q0) + b(q1)``.
    """
    kind: int
    q0: int
    q1: int = -1
    theta: float = 0.0
    phi: float = 0.0
    u: object = None

    @property
    def two_qubit(self) -> bool:
        return self.q1 >= 0


@dataclass
class Circuit:
    n_qubits: int
    gates: list
    rows: int = 0
    cols: int = 0
    depth: int = 0
    seed: int = 0

    def n_two_qubit(self) -> int:
        return sum(1 for g in self.gates if g.two_qubit)


def couplers(rows: int, cols: int, cls: str):
    """Qubit pairs (q0 < q1) of coupler class ``cls`` on a rows x cols grid."""
    out = []
    if cls in "AB":
        parity = 0 if cls == "A" else 1
        for r in range(rows):
            for c in range(cols - 1):
                if c % 2 == parity:
                    out.append((r * cols + c, r * cols + c + 1))
    else:
        parity = 0 if cls == "C" else 1
        for r in range(rows - 1):
            for c in range(cols):
                if r % 2 == parity:
                    out.append((r * cols + c, (r + 1) * cols + c))
    return out


def grid_rqc(rows: int, cols: int, depth: int, seed: int,
             theta: float = FSIM_THETA, phi: float = FSIM_PHI) -> Circuit:
    """Seeded (1+depth+1) grid random circuit (reading stated in the module doc).

    Random draws come from ``numpy.random.default_rng(seed)`` in the order
    (layer, qubit): the first draw of a qubit is uniform over three gates,
    later draws uniform over the two gates other than its previous one.
    """
    n = rows * cols
    rng = np.random.default_rng(seed)
    gates = [Gate(H, q) for q in range(n)]
    prev = [-1] * n

    def one_qubit_layer():
        for q in range(n):
            if prev[q] < 0:
                g = int(rng.integers(3))
            else:
                g = (prev[q] + 1 + int(rng.integers(2))) % 3
            prev[q] = g
            gates.append(Gate(_ONE_QUBIT_DRAWS[g], q))

    for cyc in range(depth):
        one_qubit_layer()
        for (a, b) in couplers(rows, cols, PATTERN[cyc % 8]):
            gates.append(Gate(FSIM, a, b, theta, phi))
    one_qubit_layer()
    return Circuit(n, gates, rows, cols, depth, seed)


def product_circuit(n: int, layers: int, seed: int) -> Circuit:
    """H layer followed by random single-qubit layers only (no entangling gate)."""
    rng = np.random.default_rng(seed)
    gates = [Gate(H, q) for q in range(n)]
    for _ in range(layers):
        for q in range(n):
            gates.append(Gate(_ONE_QUBIT_DRAWS[int(rng.integers(3))], q))
    return Circuit(n, gates, 1, n, 0, seed)


def random_bits(n: int, seed: int) -> np.ndarray:
    """n uniform bits (uint8) from a seeded generator."""
    return np.random.default_rng(seed).integers(0, 2, size=n, dtype=np.uint8)


def default_open_qubits(n_qubits: int, n_open: int):
    """The last ``n_open`` qubits in row-major order (the bottom row first fills)."""
    return list(range(n_qubits - n_open, n_qubits))


def bitstring_batch(n_qubits: int, open_qubits, n_batch: int, seed: int) -> np.ndarray:
    """Closed-qubit bits for ``n_batch`` requests: shape (n_batch, n_closed), uint8,
    columns in increasing qubit order of the closed qubits."""
    n_closed = n_qubits - len(open_qubits)
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, size=(n_batch, n_closed), dtype=np.uint8)


def random_complex(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """I.i.d. complex normal entries with unit variance (E|z|^2 = 1)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return ((re + 1j * im) / math.sqrt(2.0)).astype(dtype)


@dataclass
class SyntheticStep:
    """A pairwise contraction with all dimensions 2.

    ``labels_a`` etc. list the index labels of each operand from the most
    significant address bit to the least significant one (numpy C order: the
    last label has stride 1).  Shared labels absent from ``labels_c`` are
    summed.
    """
    labels_a: list
    labels_b: list
    labels_c: list
    seed: int

    @property
    def m(self):
        return len(set(self.labels_a) - set(self.labels_b))

    @property
    def n(self):
        return len(set(self.labels_b) - set(self.labels_a))

    @property
    def s(self):
        return len(set(self.labels_a) & set(self.labels_b))


def synthetic_step(rank_a: int, rank_b: int, shared: int, seed: int) -> SyntheticStep:
    """Random pair of index lists: ``shared`` contracted labels, random
    permutations of both operands and of the output."""
    rng = np.random.default_rng(seed)
    m = rank_a - shared
    n = rank_b - shared
    free_a = list(range(m))
    free_b = list(range(m, m + n))
    kk = list(range(m + n, m + n + shared))
    la = free_a + kk
    lb = kk + free_b
    lc = free_a + free_b
    la = [la[i] for i in rng.permutation(len(la))]
    lb = [lb[i] for i in rng.permutation(len(lb))]
    lc = [lc[i] for i in rng.permutation(len(lc))]
    return SyntheticStep(la, lb, lc, seed)


def synthetic_step_cases(seed: int, n_cases: int = 12, lo: int = 24, hi: int = 32,
                         s_lo: int = 8, s_hi: int = 16, max_out: int = 30):
    """Rank-24..32 pairs with 8..16 shared indices, rejecting outputs above
    2^max_out elements."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n_cases:
        ra = int(rng.integers(lo, hi + 1))
        rb = int(rng.integers(lo, hi + 1))
        s = int(rng.integers(s_lo, s_hi + 1))
        if ra + rb - 2 * s > max_out or s > min(ra, rb):
            continue
        out.append(synthetic_step(ra, rb, s, int(rng.integers(1 << 31))))
    return out


def poisson_arrivals(rate_per_s: float, n: int, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
