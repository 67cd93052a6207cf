"""Pins of the CPU oracle against things other than itself.

* gate tables vs textbook identities ((sqrt G)^2 = -iG, fSim special cases);
* hand-derived state vectors of tiny circuits (tests/golden/small_circuits.txt);
* unitarity (the squared amplitudes of all bitstrings sum to 1);
* state vector vs tensor network (two independent evaluations of <b|U|0>);
* slice sum vs unsliced contraction, and each slice vs a projector inserted
  into the state-vector simulation (Section 5.1 slicing);
* mirror circuit U^dagger U and product circuits in closed form;
* Porter-Thomas statistics of a random circuit (Section 6.2);
* the single-step oracle vs brute-force loops and vs sampled direct sums.
"""
import math
import os

import numpy as np
import pytest

import rqcgen
import oracle
from oracle import tn as otn

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "small_circuits.txt")

X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
W = (X + Y) / math.sqrt(2)
SWAP = np.eye(4)[[0, 2, 1, 3]]


def test_sqrt_gates_square_to_minus_i_g():
    for s, g in ((oracle.SQRT_X_M, X), (oracle.SQRT_Y_M, Y), (oracle.SQRT_W_M, W)):
        assert np.allclose(s @ s, -1j * g, atol=1e-15)
        assert np.allclose(s.conj().T @ s, np.eye(2), atol=1e-15)
    assert np.allclose(oracle.H_M @ oracle.H_M, np.eye(2), atol=1e-15)


def test_fsim_special_cases():
    assert np.allclose(oracle.fsim(0.0, 0.0), np.eye(4))
    phi = 0.37
    assert np.allclose(oracle.fsim(0.0, phi), np.diag([1, 1, 1, np.exp(-1j * phi)]))
    assert np.allclose(oracle.fsim(math.pi / 2, 0.0), SWAP @ np.diag([1, -1j, -1j, 1]))
    f = oracle.fsim(math.pi / 2, math.pi / 6)
    assert np.allclose(f, SWAP @ np.diag([1, -1j, -1j, np.exp(-1j * math.pi / 6)]))
    assert np.allclose(f.conj().T @ f, np.eye(4))
    # symmetric under exchange of the two qubits
    assert np.allclose(SWAP @ f @ SWAP, f)


def _golden_cases():
    cases, cur = [], None
    kinds = {"H": rqcgen.H, "SQRT_X": rqcgen.SQRT_X, "SQRT_Y": rqcgen.SQRT_Y,
             "SQRT_W": rqcgen.SQRT_W, "FSIM": rqcgen.FSIM}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "case":
            cur = {"name": tok[1], "gates": [], "amps": {}}
            cases.append(cur)
        elif tok[0] == "n":
            cur["n"] = int(tok[1])
        elif tok[0] == "gate":
            k = kinds[tok[1]]
            if k == rqcgen.FSIM:
                cur["gates"].append(rqcgen.Gate(k, int(tok[2]), int(tok[3]),
                                                float(tok[4]) * math.pi,
                                                float(tok[5]) * math.pi))
            else:
                cur["gates"].append(rqcgen.Gate(k, int(tok[2])))
        elif tok[0] == "amp":
            cur["amps"][int(tok[1])] = complex(float(tok[2]), float(tok[3]))
    return cases


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_golden_small_circuits(case):
    c = rqcgen.Circuit(case["n"], case["gates"])
    psi = oracle.statevector(c)
    want = np.zeros(1 << case["n"], dtype=complex)
    for i, v in case["amps"].items():
        want[i] = v
    assert np.allclose(psi, want, atol=1e-14)
    # the tensor network with every qubit open gives the same vector
    got = oracle.amplitudes_tn(c, list(reversed(range(case["n"]))), [])
    assert np.allclose(got, want, atol=1e-14)


def test_grid_circuit_gate_counts():
    # Coupler classes are matchings; each coupler class fires on its cycles.
    assert rqcgen.grid_rqc(4, 4, 8, 1).n_two_qubit() == 48
    assert rqcgen.grid_rqc(6, 6, 14, 2).n_two_qubit() == 210
    assert rqcgen.grid_rqc(10, 10, 20, 4).n_two_qubit() == 900
    for cls in "ABCD":
        pairs = rqcgen.couplers(6, 6, cls)
        qs = [q for p in pairs for q in p]
        assert len(qs) == len(set(qs))


def test_no_repeat_single_qubit_draws():
    c = rqcgen.grid_rqc(3, 3, 6, 9)
    last = {}
    for g in c.gates:
        if g.kind in (rqcgen.SQRT_X, rqcgen.SQRT_Y, rqcgen.SQRT_W):
            assert last.get(g.q0) != g.kind
            last[g.q0] = g.kind


def test_unitarity_statevector_and_tn():
    c = rqcgen.grid_rqc(3, 3, 6, 5)
    psi = oracle.statevector(c)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-12
    amps = oracle.amplitudes_tn(c, list(range(9)), [])
    assert abs(np.sum(np.abs(amps) ** 2) - 1.0) < 1e-12


def test_statevector_vs_tn_4x4():
    c = rqcgen.grid_rqc(4, 4, 8, 1)
    openq = [12, 13, 14, 15]
    closed = rqcgen.random_bits(12, 7)
    a_sv = oracle.amplitudes_sv(c, openq, closed)
    a_tn = oracle.amplitudes_tn(c, openq, closed)
    assert np.max(np.abs(a_sv - a_tn)) * 2 ** 8 < 1e-12
    # batch order: bit i of the batch index is open qubit openq[i]
    psi = oracle.statevector(c)
    bits = [0] * 16
    ci = 0
    for q in range(16):
        if q not in openq:
            bits[q] = int(closed[ci])
            ci += 1
    bits[openq[0]] = 1          # batch index 1
    assert abs(a_tn[1] - psi[oracle.bit_index(bits)]) < 1e-14


def test_slices_sum_to_unsliced_and_match_projectors():
    c = rqcgen.grid_rqc(4, 4, 8, 3)
    openq = [14, 15]
    closed = rqcgen.random_bits(14, 4)
    full = oracle.amplitudes_tn(c, openq, closed)
    rng = np.random.default_rng(0)
    wires = sorted(otn.wire_labels(c))
    for trial in range(3):
        pick = rng.choice(len(wires), size=4, replace=False)
        sliced = [wires[i] for i in pick]
        vals = oracle.slice_values_tn(c, openq, closed, sliced, range(16))
        assert np.max(np.abs(vals.sum(axis=0) - full)) < 1e-15
        for sid in (0, 5, 15):
            proj = {w: (sid >> j) & 1 for j, w in enumerate(sliced)}
            sv = oracle.amplitudes_sv(c, openq, closed, proj)
            assert np.max(np.abs(sv - vals[sid])) < 1e-15
    # a slice is not in general the same as the full amplitude
    assert np.max(np.abs(vals[0] - full)) > 1e-6


def _dagger(g):
    m = oracle.gate_matrix(g).conj().T
    if g.two_qubit:
        return rqcgen.Gate(rqcgen.U2, g.q0, g.q1, u=m)
    return rqcgen.Gate(rqcgen.U1, g.q0, u=m)


def test_mirror_circuit():
    c = rqcgen.grid_rqc(3, 4, 4, 11)
    mirror = rqcgen.Circuit(12, c.gates + [_dagger(g) for g in reversed(c.gates)])
    a = oracle.amplitudes_tn(mirror, [0, 5, 11], [0] * 9)
    want = np.zeros(8, dtype=complex)
    want[0] = 1.0
    assert np.max(np.abs(a - want)) < 1e-12


def test_product_circuit_closed_form():
    c = rqcgen.product_circuit(7, 5, 3)
    bits = rqcgen.random_bits(7, 2)
    per_q = []
    for q in range(7):
        v = np.array([1, 0], dtype=complex)
        for g in c.gates:
            if g.q0 == q:
                v = oracle.gate_matrix(g) @ v
        per_q.append(v)
    want = np.prod([per_q[q][bits[q]] for q in range(7)])
    got_tn = oracle.amplitudes_tn(c, [], bits)[0]
    got_sv = oracle.amplitudes_sv(c, [], bits)[0]
    assert abs(got_tn - want) < 1e-14 and abs(got_sv - want) < 1e-14


def test_porter_thomas_4x4():
    """Section 6.2: probabilities of a deep random circuit follow
    Porter-Thomas, i.e. 2^n |a|^2 is close to Exp(1)."""
    c = rqcgen.grid_rqc(4, 4, 12, 21)
    p = np.abs(oracle.statevector(c)) ** 2 * 2 ** 16
    assert abs(p.mean() - 1.0) < 1e-10
    from scipy import stats
    ks = stats.kstest(p, "expon").statistic
    assert ks < 0.02
    # a product state is far from Porter-Thomas
    q = np.abs(oracle.statevector(rqcgen.product_circuit(16, 3, 1))) ** 2 * 2 ** 16
    assert stats.kstest(q, "expon").statistic > 0.1


def test_step_einsum_vs_loops():
    rng = np.random.default_rng(1)
    la, lb, lc = [0, 1, 2, 3], [2, 4, 0], [4, 1, 3]   # K = {0, 2}
    a = rqcgen.random_complex(16, 5)
    b = rqcgen.random_complex(8, 6)
    got = oracle.einsum_step(a, b, la, lb, lc)
    A = a.reshape(2, 2, 2, 2)
    B = b.reshape(2, 2, 2)
    want = np.zeros((2, 2, 2), dtype=complex)
    for x4 in range(2):
        for x1 in range(2):
            for x3 in range(2):
                s = 0
                for x0 in range(2):
                    for x2 in range(2):
                        s += A[x0, x1, x2, x3] * B[x2, x4, x0]
                want[x4, x1, x3] = s
    assert np.allclose(got, want.reshape(-1), atol=1e-14)
    del rng


def test_step_gemm_shape_vs_matmul():
    a = rqcgen.random_complex(2 ** 7, 1)
    b = rqcgen.random_complex(2 ** 6, 2)
    # A[m(3 bits), k(4 bits)], B[k(4 bits)... only 2 free]: C = A @ B
    la = [0, 1, 2, 10, 11, 12, 13]
    lb = [10, 11, 12, 13, 20, 21]
    lc = [0, 1, 2, 20, 21]
    got = oracle.einsum_step(a, b, la, lb, lc)
    want = a.reshape(8, 16) @ b.reshape(16, 4)
    assert np.allclose(got, want.reshape(-1), atol=1e-13)


def test_sampled_step_vs_einsum():
    st = rqcgen.synthetic_step(9, 8, 4, 77)
    a = rqcgen.random_complex(1 << 9, 3)
    b = rqcgen.random_complex(1 << 8, 4)
    full = oracle.einsum_step(a, b, st.labels_a, st.labels_b, st.labels_c)
    coords = np.random.default_rng(2).integers(0, full.size, size=40)
    got = oracle.sampled_step(lambda i: a[i], lambda i: b[i],
                              st.labels_a, st.labels_b, st.labels_c, coords)
    assert np.allclose(got, full[coords], atol=1e-13)


def test_metrics():
    ref = np.array([1 + 1j, 2, -1j]) / 8
    assert oracle.normalized_error(ref, ref, 6) == 0
    assert abs(oracle.normalized_error(ref + 1 / 8, ref, 6) - 1.0) < 1e-15
    assert abs(oracle.linear_fidelity(3j * ref, ref) - 1.0) < 1e-15
    assert oracle.linear_fidelity(np.array([1, 0]), np.array([0, 1])) == 0.0
    # Hand-computed values.  ref = (1, 2, 0), got = (1+1j, 2, 0.5):
    # |got - ref| = (1, 0, 0.5), max 1; RMS(ref) = sqrt(5/3).
    r3 = np.array([1, 2, 0], dtype=complex)
    g3 = np.array([1 + 1j, 2, 0.5])
    assert abs(oracle.per_slice_error(g3, r3) - 0.7745966692414834) < 1e-15  # sqrt(3/5)
    # Natural scale of a 4-qubit amplitude cut on 2 wires: 2^-3.  A tiny
    # reference (RMS 1e-30) is measured against it: 0.01 / 0.125.
    assert oracle.natural_slice_scale(4, 2) == 0.125
    tiny = np.array([1e-30, -1e-30j])
    assert abs(oracle.slice_error_natural(tiny + 0.01, tiny, 4, 2) - 0.08) < 1e-15
    # Above the natural scale it is the error relative to the RMS.
    assert abs(oracle.slice_error_natural(g3, r3, 4, 2) - 0.7745966692414834) < 1e-15
    assert abs(oracle.slice_error_natural(g3 * 0.5, r3 * 0.5, 2, 0) - 0.7745966692414834) < 1e-15
    # With the 2^-(n+S)/2 scale above the RMS: n = 0, S = 0 gives 1.
    assert abs(oracle.slice_error_natural(r3 * 1e-3 + 1e-3, r3 * 1e-3, 0, 0) - 1e-3) < 1e-15


def test_linear_xeb():
    # Hand-computed: amplitudes (0.6, 0.8) of one qubit, p = (0.36, 0.64).
    a = np.array([0.6, 0.8j])
    assert abs(oracle.xeb_ideal_sampling(a, 1) - 0.0784) < 1e-15   # 2 * 0.5392 - 1
    assert abs(oracle.xeb_of_samples(a, 1, [1, 1, 0]) - 0.09333333333333327) < 1e-15
    assert abs(oracle.xeb_of_samples(a, 1, [0, 1])) < 1e-15       # every entry once
    # Uniform amplitudes: 0; a basis state: 2^n - 1.
    u = np.full(16, 0.25)
    assert abs(oracle.xeb_ideal_sampling(u, 4)) < 1e-15
    d = np.zeros(8)
    d[5] = 1.0
    assert oracle.xeb_ideal_sampling(d, 3) == 7.0
    assert oracle.xeb_of_samples(d, 3, [5]) == 7.0
    # Porter-Thomas (Section 6.2): for a random circuit 2^n sum p^2 is close
    # to 2, so ideal sampling scores about 1.
    c = rqcgen.grid_rqc(4, 4, 12, 3)
    psi = oracle.statevector(c)
    assert abs(oracle.xeb_ideal_sampling(psi, 16) - 1.0) < 0.1


def _random_order(tensors, rng):
    """A random grouping of the tensors and a random tree over the groups:
    each pair is drawn among the three connected pairs with the fewest
    result labels, so intermediates stay small."""
    idx = list(rng.permutation(len(tensors)))
    groups = []
    while idx:
        k = int(rng.integers(1, 4))
        groups.append([int(i) for i in idx[:k]])
        idx = idx[k:]
    labels = {g: set(l for i in m for l in tensors[i][1]) for g, m in enumerate(groups)}
    live = dict(labels)
    pairs = []
    nid = len(groups)
    while len(live) > 1:
        keys = list(live)
        cand = sorted((len(live[a] ^ live[b]), a, b) for a in keys for b in keys
                      if a < b and live[a] & live[b])
        if cand:
            _, a, b = cand[int(rng.integers(min(3, len(cand))))]
        else:
            a, b = keys[0], keys[1]
        pairs.append((a, b))
        live[nid] = live.pop(a) | live.pop(b)
        nid += 1
    return groups, pairs


def test_contract_ordered_vs_statevector_random_trees():
    """Any order given as data reaches the same amplitudes: random groupings
    and random trees vs the state vector, with and without slicing."""
    rng = np.random.default_rng(3)
    c = rqcgen.grid_rqc(2, 3, 5, 8)
    openq = [4, 5]
    closed = rqcgen.random_bits(4, 2)
    ref = oracle.amplitudes_sv(c, openq, closed)
    for _ in range(4):
        tensors, out = otn.build_network(c, openq, closed)
        groups, pairs = _random_order(tensors, rng)
        got = oracle.contract_ordered(tensors, out, groups, pairs)
        assert np.max(np.abs(got - ref)) < 1e-14
    wires = sorted(otn.wire_labels(c))
    sliced = [wires[i] for i in rng.choice(len(wires), size=3, replace=False)]
    tensors, _ = otn.build_network(c, openq, closed, sliced, 0)
    groups, pairs = _random_order(tensors, rng)
    vals = oracle.slice_values_ordered(c, openq, closed, sliced, range(8), groups, pairs)
    assert np.max(np.abs(vals.sum(axis=0) - ref)) < 1e-14
    for sid in (0, 6):
        proj = {w: (sid >> j) & 1 for j, w in enumerate(sliced)}
        assert np.max(np.abs(oracle.amplitudes_sv(c, openq, closed, proj) - vals[sid])) < 1e-14


def test_contract_ordered_rejects_bad_groups():
    c = rqcgen.grid_rqc(2, 2, 2, 1)
    tensors, out = otn.build_network(c, [0], [0, 1, 1])
    with pytest.raises(ValueError):
        oracle.contract_ordered(tensors, out, [[0, 1]], [])


def test_ttgt_example_section_5_4():
    """The worked example of Section 5.4: A[a,b,c,d,e,f,g] (7 indices) and
    B[h,a,f,i] contracted over {a,f} into C[b,c,d,e,g,h,i].  The paper's
    procedure -- B permuted to B^T[a,f,h,i], A permuted so that the kept
    indices come first and the summed ones last, one matrix product, the
    result in the order of C -- done here with numpy transposes and a matrix
    product, must equal the oracle's single step (einsum)."""
    a, b, c, d, e, f, g, h, i = range(9)
    rng = np.random.default_rng(54)
    A = rng.standard_normal(2 ** 7) + 1j * rng.standard_normal(2 ** 7)
    B = rng.standard_normal(2 ** 4) + 1j * rng.standard_normal(2 ** 4)
    la, lb, lc = [a, b, c, d, e, f, g], [h, a, f, i], [b, c, d, e, g, h, i]
    At = A.reshape((2,) * 7).transpose(1, 2, 3, 4, 6, 0, 5).reshape(2 ** 5, 2 ** 2)  # [bcdeg | af]
    Bt = B.reshape((2,) * 4).transpose(1, 2, 0, 3).reshape(2 ** 2, 2 ** 2)            # [af | hi]
    C = (At @ Bt).reshape(-1)                                                          # [bcdeg hi]
    ref = oracle.einsum_step(A, B, la, lb, lc)
    assert np.max(np.abs(C - ref)) < 1e-13
    # and an index-by-index sum for one entry
    cb, cc, cd, ce, cg, ch, ci = 1, 0, 1, 1, 0, 1, 0
    direct = sum(A.reshape((2,) * 7)[ka, cb, cc, cd, ce, kf, cg] * B.reshape((2,) * 4)[ch, ka, kf, ci]
                 for ka in (0, 1) for kf in (0, 1))
    idx = int("".join(map(str, (cb, cc, cd, ce, cg, ch, ci))), 2)
    assert abs(ref[idx] - direct) < 1e-13
