"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (FP32 path): amplitudes normalised by the RMS amplitude
2^(-n/2) must agree to 1e-4; single contraction steps to max(2e-5, 6 u sqrt(K))
relative to the RMS of the reference.  The rounding of a K-term FP32 sum of
random-sign products grows like u sqrt(K) relative to the RMS output
(u = 2^-24, partial sums growing as a random walk); the three-product form
of the complex product (Im C = P3 - P1 - P2) roughly doubles it, and the
factor 6 covers a 4-sigma tail over the checked outputs.  For the sums of
up to 2^9 terms of most cases this is 2e-5; for the rank-24..32 steps with
up to 2^16 summed terms it reaches 9e-5.
Reduced precision: normalised error <= 2e-2 and linear fidelity >= 0.99.
"""
import sys

import numpy as np
import pytest

import rqcgen
import oracle
from plan_order import oracle_order, oracle_wires_and_ids

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2110_14502_amd")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _dev_c64(x):
    return torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64))).cuda()


def fp32_step_tol(k_bits):
    """Single-step FP32 bound for sums of 2^k_bits terms (module docstring)."""
    return max(2e-5, 6 * 2.0 ** -24 * 2.0 ** (k_bits / 2))


def _rel_rms(got, ref):
    ref = np.asarray(ref)
    return float(np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2)))


# ---------------------------------------------------------------- single steps
STEP_CASES = [
    # (rank_a, rank_b, shared, seed, kernel)
    (12, 10, 5, 1, 0),
    (9, 4, 2, 2, 0),     # imbalanced: big A, small B
    (14, 12, 5, 3, 1),   # MFMA: m=9, n=7, k=5
    (16, 13, 7, 4, 1),
    (15, 15, 4, 5, -1),
    (6, 6, 6, 6, 0),     # full contraction to a scalar
    (5, 3, 0, 7, 0),     # outer product
    (18, 16, 9, 8, 1),   # long sum: one tile per workgroup (k >= 8)
    (17, 17, 8, 9, -1),
    (15, 15, 12, 10, 0),  # 8 x 8 output, long sum: blocked tiny-tile form
    (14, 13, 11, 11, 0),  # 8 x 4 output
]


@pytest.mark.parametrize("ra,rb,s,seed,kernel", STEP_CASES)
def test_pair_contract_vs_einsum(ra, rb, s, seed, kernel):
    _say("pair", ra, rb, s, seed, kernel)
    st = rqcgen.synthetic_step(ra, rb, s, seed)
    a = rqcgen.random_complex(1 << ra, seed + 100)
    b = rqcgen.random_complex(1 << rb, seed + 200)
    ref = oracle.einsum_step(a, b, st.labels_a, st.labels_b, st.labels_c)
    c = R.pair_contract(_dev_c64(a), _dev_c64(b), st.labels_a, st.labels_b, st.labels_c,
                        kernel=kernel)
    torch.cuda.synchronize()
    got = c.cpu().numpy().astype(np.complex128)
    assert _rel_rms(got, ref) < 2e-5


def test_pair_contract_batched_and_shared_operand():
    _say("pair batched")
    st = rqcgen.synthetic_step(13, 11, 5, 9)
    nb = 3
    a = rqcgen.random_complex((nb, 1 << 13), 11)
    b = rqcgen.random_complex(1 << 11, 12)  # shared by every batch entry
    c = R.pair_contract(_dev_c64(a), _dev_c64(b), st.labels_a, st.labels_b, st.labels_c,
                        batch=nb, stride_a=1 << 13, stride_b=0, kernel=1)
    torch.cuda.synchronize()
    got = c.cpu().numpy().reshape(nb, -1)
    for i in range(nb):
        ref = oracle.einsum_step(a[i], b, st.labels_a, st.labels_b, st.labels_c)
        assert _rel_rms(got[i], ref) < 2e-5


def test_permute_and_cgemm():
    _say("permute cgemm")
    rng = np.random.default_rng(3)
    r = 14
    lin = list(range(r))
    lout = [lin[i] for i in rng.permutation(r)]
    x = rqcgen.random_complex(1 << r, 4)
    y = R.permute(_dev_c64(x), lin, lout)
    torch.cuda.synchronize()
    ref = oracle.einsum_step(x, np.ones(1), lin, [], lout)
    assert np.array_equal(y.cpu().numpy(), ref.astype(np.complex64))
    M, N, K = 256, 128, 64
    A = rqcgen.random_complex(M * K, 5)
    B = rqcgen.random_complex(K * N, 6)
    Cg = R.cgemm(_dev_c64(A), _dev_c64(B), M, N, K)
    torch.cuda.synchronize()
    ref = A.reshape(M, K) @ B.reshape(K, N)
    assert _rel_rms(Cg.cpu().numpy().reshape(M, N), ref) < 2e-5


# ---------------------------------------------------------------- amplitudes
def _setup(rows, cols, depth, cseed, n_open, **kw):
    c = rqcgen.grid_rqc(rows, cols, depth, cseed)
    n = rows * cols
    openq = list(range(n - n_open, n))
    P = R.Plan(R.Network(R.Circuit.from_rqcgen(c), openq), **kw).bind()
    return c, openq, P


def test_config1_single_amplitude_vs_statevector():
    """4x4 grid, depth 1+8+1, greedy path, no slicing, one bitstring."""
    _say("config1")
    c, openq, P = _setup(4, 4, 8, 1, 0, seed=1)
    bits = rqcgen.random_bits(16, 1)
    got = R.to_complex(P.contract(bits))[0]
    ref = oracle.amplitudes_sv(c, [], bits)
    assert oracle.normalized_error(got, ref, 16) < 1e-4
    # and with four open qubits (a batch of 16 amplitudes)
    c, openq, P = _setup(4, 4, 8, 1, 4, seed=1)
    got = R.to_complex(P.contract(bits[:12]))[0]
    ref = oracle.amplitudes_sv(c, openq, bits[:12])
    assert oracle.normalized_error(got, ref, 16) < 1e-4
    assert oracle.linear_fidelity(got, ref) > 0.999999


def test_all_qubits_open_is_normalised():
    _say("all open")
    c, openq, P = _setup(3, 4, 6, 2, 12, seed=3)
    got = R.to_complex(P.contract(np.zeros(0, np.uint8)))[0]
    assert abs(np.sum(np.abs(got) ** 2) - 1.0) < 1e-5
    ref = oracle.amplitudes_sv(c, openq, [])
    assert oracle.normalized_error(got, ref, 12) < 1e-4


def _sliced_case(prec, n_sliced=5, depth=8, cseed=3):
    c, openq, P = _setup(5, 5, depth, cseed, 4, n_sliced=n_sliced, seed=5, path_trials=64)
    bits = rqcgen.random_bits(21, 9)
    wires = P.sliced_wires()
    amps, per = P.contract(bits, prec=prec, per_slice=True)
    ref_slices = oracle.slice_values_tn(c, openq, bits, wires, range(1 << n_sliced))
    return c, P, bits, R.to_complex(amps)[0], R.to_complex(per)[:, 0], ref_slices


def test_sliced_per_slice_and_sum_fp32():
    _say("sliced fp32")
    c, P, bits, amps, per, ref = _sliced_case(R.F32)
    assert per.shape == ref.shape
    err = oracle.per_slice_error(per, ref)
    assert err < 1e-4
    full = oracle.amplitudes_tn(c, list(range(21, 25)), bits)
    assert np.max(np.abs(ref.sum(0) - full)) < 1e-13  # oracle self-consistency
    assert oracle.normalized_error(amps, full, 25) < 1e-4


def _lp_case():
    """5x5 (1+12+1), four open qubits, four sliced wires, FP16 storage from
    2^6 and BF16 storage from 2^10 elements per slice (BF16 keeps 8
    significand bits and rounds more per stored stage; the library default
    is 2^24): the plan has 16-bit matrix-core steps and 16-bit stored
    intermediates on the slice-dependent path."""
    c = rqcgen.grid_rqc(5, 5, 12, 3)
    openq = [21, 22, 23, 24]
    P = R.Plan(R.Network(R.Circuit.from_rqcgen(c), openq), n_sliced=4, seed=5, path_trials=64,
               lp_min_log2=6, bf16_min_log2=10).bind()
    bits = rqcgen.random_bits(21, 9)
    e = P.export()
    groups, pairs = oracle_order(c, openq, e)
    ow, oids = oracle_wires_and_ids(e, range(16))
    ref = oracle.slice_values_ordered(c, openq, bits, ow, oids, groups, pairs)
    return c, P, bits, ref


@pytest.fixture(scope="module")
def lp_case():
    return _lp_case()


def test_lp_case_plan_runs_16_bit_work(lp_case):
    _, P, _, _ = lp_case
    st = [s for s in P.steps() if s["depends_on_slice"]]
    assert sum(s["kernel_lp"] == R.KERN_MFMA16 for s in st) >= 4
    assert sum(s["lp_output"] for s in st) >= 10
    assert sum(s["lp_output_bf16"] for s in st) >= 10


def test_lp_case_fp32_vs_oracle(lp_case):
    _say("lp case fp32")
    _, P, bits, ref = lp_case
    amps, per = P.contract(bits, per_slice=True)
    assert oracle.slice_error_natural(R.to_complex(per)[:, 0], ref, 25, 4) < 1e-4
    assert oracle.normalized_error(R.to_complex(amps)[0], ref.sum(0), 25) < 1e-4


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_lp_case_reduced_precision_vs_oracle(lp_case, prec):
    """Amplitudes and slices of a plan whose 16-bit paths run, against the
    oracle: normalised error <= 2e-2, linear fidelity >= 0.99, and above the
    FP32 level (the 16-bit path ran)."""
    _say("lp case", prec)
    _, P, bits, ref = lp_case
    amps, per = P.contract(bits, prec=R.PRECISIONS[prec], per_slice=True)
    amps = R.to_complex(amps)[0]
    per = R.to_complex(per)[:, 0]
    full = ref.sum(0)
    err = oracle.normalized_error(amps, full, 25)
    assert 1e-6 < err < 2e-2, err
    assert oracle.linear_fidelity(amps, full) > 0.99
    assert oracle.slice_error_natural(per, ref, 25, 4) < 2e-2
    assert oracle.linear_fidelity(per, ref) > 0.99
    assert P.last_report["fp32_reruns"] == 0


def test_overflow_filter_reruns_in_fp32():
    """Section 5.5 filter: a forced overflow flags every slice, which is then
    recomputed in FP32 (the host forces it through a storage-exponent bias;
    the kernels themselves run normally)."""
    _say("rerun")
    c, openq, P = _setup(5, 5, 8, 3, 4, n_sliced=3, seed=5, path_trials=32, lp_min_log2=4)
    bits = rqcgen.random_bits(21, 9)
    P.set_scale_bias(40)
    amps = R.to_complex(P.contract(bits, prec=R.F16))[0]
    assert P.last_report["fp32_reruns"] == 8
    full = oracle.amplitudes_tn(c, openq, bits)
    assert oracle.normalized_error(amps, full, 25) < 1e-4
    P.set_scale_bias(0)


def test_overflow_in_later_bitstring_groups_is_rerun_once():
    """The filter with one bitstring per group and the overflow forced only
    from the second bitstring on: the first bitstring keeps its FP16 sum,
    the others get exactly one FP32 copy of every slice (none is counted
    twice), and the per-slice rows of the re-run groups are the FP32 ones."""
    _say("rerun later groups")
    c, openq, P = _setup(5, 5, 8, 3, 4, n_sliced=3, seed=5, path_trials=32, lp_min_log2=4)
    bits = np.stack([rqcgen.random_bits(21, s) for s in (9, 10, 11)])
    P.set_group_limit(0, 1)
    P.set_scale_bias(40, first_bitstring=1)
    amps, per = P.contract(bits, prec=R.F16, per_slice=True)
    assert P.last_report["bits_per_group"] == 1
    assert P.last_report["fp32_reruns"] == 8
    amps, per = R.to_complex(amps), R.to_complex(per)
    wires = P.sliced_wires()
    for i in range(3):
        ref = oracle.slice_values_tn(c, openq, bits[i], wires, range(8))
        full = ref.sum(0)
        err = oracle.normalized_error(amps[i], full, 25)
        if i == 0:
            assert 1e-6 < err < 2e-2, err  # FP16, not re-run
        else:
            assert err < 1e-4, (i, err)   # FP32 re-run, added once
            assert oracle.per_slice_error(per[:, i], ref) < 1e-4
    P.set_scale_bias(0)
    P.set_group_limit(0, 0)


def test_graph_replay_is_bitwise_identical():
    _say("graph replay")
    c, openq, P = _setup(5, 5, 8, 3, 4, n_sliced=4, seed=5, path_trials=32)
    bits = rqcgen.random_bits(21, 9)
    a1 = P.contract(bits).clone()
    r1 = P.last_report
    a2 = P.contract(bits).clone()
    r2 = P.last_report
    assert r1["graph_reused"] == 0 and r2["graph_reused"] == 1
    assert torch.equal(a1, a2)
    # different closed bits through the same graph
    bits2 = rqcgen.random_bits(21, 10)
    a3 = R.to_complex(P.contract(bits2))[0]
    assert P.last_report["graph_reused"] == 1
    ref = oracle.amplitudes_tn(c, openq, bits2)
    assert oracle.normalized_error(a3, ref, 25) < 1e-4


def test_bitstring_batch_and_slice_subsets_and_small_workspace():
    _say("batch subsets")
    c, openq, P = _setup(5, 5, 8, 3, 4, n_sliced=4, seed=5, path_trials=32)
    bits = np.stack([rqcgen.random_bits(21, s) for s in (1, 2, 3)])
    batch = R.to_complex(P.contract(bits))
    for i in range(3):
        ref = oracle.amplitudes_tn(c, openq, bits[i])
        assert oracle.normalized_error(batch[i], ref, 25) < 1e-4
    # a subset of slices, with a workspace that forces ragged groups
    ids = [0, 3, 5, 6, 9, 12, 15]
    lo, pref = P.workspace_bytes(len(ids), 1, R.F32)
    ws = torch.empty(lo + (pref - lo) // 3, dtype=torch.uint8, device="cuda")
    sub, per = P.contract(bits[0], slice_ids=ids, workspace=ws, per_slice=True)
    assert P.last_report["slices_per_group"] < len(ids)
    wires = P.sliced_wires()
    ref = oracle.slice_values_tn(c, openq, bits[0], wires, ids)
    assert oracle.per_slice_error(R.to_complex(per)[:, 0], ref) < 1e-4
    assert oracle.normalized_error(R.to_complex(sub)[0], ref.sum(0), 25) < 1e-4


def test_row_streaming_kernel_plan_layout():
    """Row-streaming kernel on a plan-style layout: summed labels lowest in
    both operands in the same order, small B, several row tiles."""
    _say("rows kernel")
    for (m, n, k, seed) in ((14, 3, 3, 21), (12, 6, 5, 22), (9, 0, 2, 23), (13, 2, 0, 24),
                            (12, 5, 7, 25), (11, 4, 6, 26),  # B of 4096 / 1024 elements
                            (12, 4, 8, 27), (10, 3, 9, 28), (9, 2, 10, 29)):  # sums of 256-1024
        M = list(range(m))
        N = list(range(100, 100 + n))
        K = list(range(200, 200 + k))
        rng = np.random.default_rng(seed)
        la = [M[i] for i in rng.permutation(m)] + K
        lb = [N[i] for i in rng.permutation(n)] + K
        lc = [x for x in (M + N)]
        lc = [lc[i] for i in rng.permutation(len(lc))]
        a = rqcgen.random_complex(1 << (m + k), seed)
        b = rqcgen.random_complex(1 << (n + k), seed + 1)
        ref = oracle.einsum_step(a, b, la, lb, lc)
        c = R.pair_contract(_dev_c64(a), _dev_c64(b), la, lb, lc, kernel=2)
        torch.cuda.synchronize()
        assert _rel_rms(c.cpu().numpy(), ref) < 2e-5, (m, n, k)


def test_dot_kernel_tiny_outputs_long_sums():
    """Tiny outputs (up to 8 x 8) with long sums whose indices are the lowest
    address bits of both operands in the same order: the streaming dot
    kernel with split sums (a workspace of partial outputs, added in split
    order), against einsum; a batch with per-copy A and shared B; and the
    same shapes with the summed indices not lowest (generic kernel)."""
    _say("dot kernel")
    for (m, n, k, batch, seed, lowest) in ((3, 3, 18, 2, 141, True), (2, 3, 16, 1, 142, True),
                                           (3, 0, 17, 3, 143, True), (1, 1, 14, 1, 144, True),
                                           (3, 3, 16, 1, 145, False)):
        M = list(range(m))
        N = list(range(100, 100 + n))
        K = list(range(200, 200 + k))
        rng = np.random.default_rng(seed)
        la = [M[i] for i in rng.permutation(m)] + K
        lb = [N[i] for i in rng.permutation(n)] + K
        if not lowest:
            la = la[m + 2:] + la[:m + 2]
        lc = [x for x in (M + N)]
        lc = [lc[i] for i in rng.permutation(len(lc))]
        need = R.pair_workspace_bytes(la, lb, lc, -1, batch, 1 << (m + k), 0, R.F32)
        assert need >= 8 * (batch << (m + n)) * 2, (m, n, k, need)
        a = rqcgen.random_complex(batch << (m + k), seed).reshape(batch, -1)
        b = rqcgen.random_complex(1 << (n + k), seed + 1)
        c = R.pair_contract(_dev_c64(a.reshape(-1)), _dev_c64(b), la, lb, lc, batch=batch,
                            stride_a=1 << (m + k), stride_b=0)
        torch.cuda.synchronize()
        got = c.cpu().numpy().reshape(batch, -1)
        for i in range(batch):
            ref = oracle.einsum_step(a[i], b, la, lb, lc)
            assert _rel_rms(got[i], ref) < fp32_step_tol(k), (m, n, k, i, lowest)


def test_row_streaming_kernel_wide_outputs():
    """Row-streaming kernel on 64- and 128-column outputs with sums of at
    most 16: the columns are walked in groups of 32 with the rows held in
    registers.  Full and partial row tiles, every sum length up to 16, and a
    batch of copies with a shared B."""
    _say("rows kernel wide")
    for (m, n, k, seed) in ((12, 6, 4, 121), (13, 7, 4, 122), (9, 7, 2, 123), (7, 6, 3, 124),
                            (10, 7, 0, 125), (11, 7, 1, 126)):
        M = list(range(m))
        N = list(range(100, 100 + n))
        K = list(range(200, 200 + k))
        rng = np.random.default_rng(seed)
        la = [M[i] for i in rng.permutation(m)] + K
        lb = [N[i] for i in rng.permutation(n)] + K
        lc = [x for x in (M + N)]
        lc = [lc[i] for i in rng.permutation(len(lc))]
        batch = 3 if seed == 122 else 1
        a = rqcgen.random_complex(batch << (m + k), seed).reshape(batch, -1)
        b = rqcgen.random_complex(1 << (n + k), seed + 1)
        c = R.pair_contract(_dev_c64(a.reshape(-1)), _dev_c64(b), la, lb, lc, kernel=2,
                            batch=batch, stride_a=1 << (m + k), stride_b=0)
        torch.cuda.synchronize()
        got = c.cpu().numpy().reshape(batch, -1)
        for i in range(batch):
            ref = oracle.einsum_step(a[i], b, la, lb, lc)
            assert _rel_rms(got[i], ref) < 2e-5, (m, n, k, i)


@pytest.mark.parametrize("prec,tol", [("f16", 6e-3), ("bf16", 4e-2)])
def test_lp_mfma_kernel_vs_einsum(prec, tol):
    """FP16 / BF16 matrix-core contraction: operands rounded to 16 bits
    (unit roundoff 2^-11 / 2^-8), FP32 accumulation.  Error relative to the
    RMS output <= a few unit roundoffs (random-sign sums keep the relative
    error at the operand rounding level)."""
    _say("lp mfma", prec)
    for (ra, rb, s, seed) in ((15, 13, 6, 31), (16, 14, 7, 32)):
        st = rqcgen.synthetic_step(ra, rb, s, seed)
        a = rqcgen.random_complex(1 << ra, seed)
        b = rqcgen.random_complex(1 << rb, seed + 1)
        ref = oracle.einsum_step(a, b, st.labels_a, st.labels_b, st.labels_c)
        c = R.pair_contract(_dev_c64(a), _dev_c64(b), st.labels_a, st.labels_b, st.labels_c,
                            prec=R.PRECISIONS[prec])
        torch.cuda.synchronize()
        got = c.cpu().numpy().astype(np.complex128)
        err = _rel_rms(got, ref)
        assert err < tol, err
        # and it is not the FP32 path: the error is at the 16-bit level
        assert err > 1e-6


@pytest.mark.parametrize("prec,tol", [("f16", 6e-3), ("bf16", 4e-2)])
def test_lp_mfma_short_sum_vs_einsum(prec, tol):
    """FP16 / BF16 matrix-core contraction of a sum of 16 (half of the
    kernel's chunk) on the planner's layout: summed labels lowest in both
    operands, in the same order."""
    _say("lp mfma short sum", prec)
    for (m, n, k, seed) in ((10, 8, 4, 41), (9, 7, 4, 42)):
        M, N, K = list(range(m)), list(range(100, 100 + n)), list(range(200, 200 + k))
        rng = np.random.default_rng(seed)
        la = [M[i] for i in rng.permutation(m)] + K
        lb = [N[i] for i in rng.permutation(n)] + K
        lc = [x for x in (M + N)]
        lc = [lc[i] for i in rng.permutation(len(lc))]
        a = rqcgen.random_complex(1 << (m + k), seed)
        b = rqcgen.random_complex(1 << (n + k), seed + 1)
        ref = oracle.einsum_step(a, b, la, lb, lc)
        c = R.pair_contract(_dev_c64(a), _dev_c64(b), la, lb, lc, prec=R.PRECISIONS[prec])
        torch.cuda.synchronize()
        err = _rel_rms(c.cpu().numpy().astype(np.complex128), ref)
        assert err < tol, (m, n, k, err)
        assert err > 1e-6  # the 16-bit path ran



@pytest.mark.parametrize("prec,tol", [("f16", 6e-3), ("bf16", 4e-2)])
def test_lp_long_sum_two_phase_vs_einsum(prec, tol):
    """Long sums in FP16 / BF16 take the two-phase form (operands permuted
    and converted into plain 16-bit matrices, then the 256 x 128-tile
    matrix-core GEMM writing C in its own layout): random index orders of A,
    B and C; one tile, several tiles in the XCD-aware order, and a batch of
    two with a shared B; sums split 2 and 8 ways over one output tile."""
    for (ra, rb, s, seed) in ((16, 15, 8, 51), (18, 16, 8, 52), (19, 17, 9, 53),
                              (18, 17, 10, 58), (20, 19, 12, 59)):
        _say("lp long sum", prec, ra, rb, s)
        st = rqcgen.synthetic_step(ra, rb, s, seed)
        assert R.pair_workspace_bytes(st.labels_a, st.labels_b, st.labels_c,
                                      prec=R.PRECISIONS[prec]) > 0
        a = rqcgen.random_complex(1 << ra, seed)
        b = rqcgen.random_complex(1 << rb, seed + 1)
        ref = oracle.einsum_step(a, b, st.labels_a, st.labels_b, st.labels_c)
        c = R.pair_contract(_dev_c64(a), _dev_c64(b), st.labels_a, st.labels_b, st.labels_c,
                            prec=R.PRECISIONS[prec])
        torch.cuda.synchronize()
        err = _rel_rms(c.cpu().numpy().astype(np.complex128), ref)
        assert err < tol, (ra, rb, s, err)
        assert err > 1e-6  # 16-bit operands
    # batch of two copies of B (stride), one shared A (stride 0)
    _say("lp long sum batch, shared A", prec)
    st = rqcgen.synthetic_step(16, 16, 8, 60)
    ra, rb, rc = len(st.labels_a), len(st.labels_b), len(st.labels_c)
    a = rqcgen.random_complex(1 << ra, 61)
    b = np.concatenate([rqcgen.random_complex(1 << rb, 62), rqcgen.random_complex(1 << rb, 63)])
    c = R.pair_contract(_dev_c64(a), _dev_c64(b), st.labels_a, st.labels_b, st.labels_c, batch=2,
                        stride_a=0, stride_b=1 << rb, prec=R.PRECISIONS[prec])
    torch.cuda.synchronize()
    got = c.cpu().numpy().astype(np.complex128)
    for j in range(2):
        ref = oracle.einsum_step(a, b[j << rb:(j + 1) << rb], st.labels_a, st.labels_b,
                                 st.labels_c)
        err = _rel_rms(got[j << rc:(j + 1) << rc], ref)
        assert 1e-6 < err < tol, (j, err)
    # batch of two copies of A (stride), one shared B (stride 0)
    _say("lp long sum batch", prec)
    st = rqcgen.synthetic_step(17, 15, 8, 54)
    ra, rb, rc = len(st.labels_a), len(st.labels_b), len(st.labels_c)
    a = np.concatenate([rqcgen.random_complex(1 << ra, 55), rqcgen.random_complex(1 << ra, 56)])
    b = rqcgen.random_complex(1 << rb, 57)
    c = R.pair_contract(_dev_c64(a), _dev_c64(b), st.labels_a, st.labels_b, st.labels_c, batch=2,
                        stride_a=1 << ra, stride_b=0, prec=R.PRECISIONS[prec])
    torch.cuda.synchronize()
    got = c.cpu().numpy().astype(np.complex128)
    for j in range(2):
        ref = oracle.einsum_step(a[j << ra:(j + 1) << ra], b, st.labels_a, st.labels_b,
                                 st.labels_c)
        err = _rel_rms(got[j << rc:(j + 1) << rc], ref)
        assert 1e-6 < err < tol, (j, err)


def test_config3_full_rank_steps_sampled():
    """Two of the rank-24..32 synthetic steps at full size (random index
    orders of both operands and the output), 256 sampled outputs each vs
    direct complex128 sums."""
    cases = rqcgen.synthetic_step_cases(3, n_cases=2)
    for i, st in enumerate(cases):
        la, lb, lc = st.labels_a, st.labels_b, st.labels_c
        k = len([x for x in la if x in lb])
        _say("config3 step", len(la), len(lb), k)
        g = torch.Generator(device="cuda").manual_seed(11 + i)
        A = torch.randn(1 << len(la), dtype=torch.complex64, device="cuda", generator=g)
        B = torch.randn(1 << len(lb), dtype=torch.complex64, device="cuda", generator=g)
        C = R.pair_contract(A, B, la, lb, lc)
        torch.cuda.synchronize()
        coords = np.random.default_rng(20 + i).integers(0, 1 << len(lc), size=256)

        def get(T):
            return lambda idx: T[torch.from_numpy(np.asarray(idx)).cuda()].cpu().numpy()
        ref = oracle.sampled_step(get(A), get(B), la, lb, lc, coords)
        got = C[torch.from_numpy(coords).cuda()].cpu().numpy()
        scale = np.sqrt(2.0 ** k)  # RMS of a sum of 2^k unit-variance products
        assert np.max(np.abs(got - ref)) / scale < fp32_step_tol(k)
        # FP16: the two-phase long-sum form (operand rounding 2^-11 per
        # component; the relative error of the sum stays near 2 u)
        C16 = R.pair_contract(A, B, la, lb, lc, prec=R.F16)
        torch.cuda.synchronize()
        got16 = C16[torch.from_numpy(coords).cuda()].cpu().numpy()
        err16 = np.max(np.abs(got16 - ref)) / scale
        assert 1e-6 < err16 < 6e-3, err16
        del A, B, C, C16


def test_ttgt_example_section_5_4_on_the_gpu():
    """Section 5.4's example contraction (A[a,b,c,d,e,f,g] B[h,a,f,i] over
    {a,f} into C[b,c,d,e,g,h,i]) with the permutation folded into the
    kernel's loads and stores, as given and with five more free indices on
    each side (several tiles; with two summed indices the generic kernel
    serves every request), against einsum."""
    _say("ttgt example")
    a, b, c, d, e, f, g, h, i = range(9)
    la, lb, lc = [a, b, c, d, e, f, g], [h, a, f, i], [b, c, d, e, g, h, i]
    x = rqcgen.random_complex(1 << 7, 54)
    y = rqcgen.random_complex(1 << 4, 55)
    ref = oracle.einsum_step(x, y, la, lb, lc)
    for kernel in (0, -1):
        got = R.pair_contract(_dev_c64(x), _dev_c64(y), la, lb, lc, kernel=kernel)
        torch.cuda.synchronize()
        assert _rel_rms(got.cpu().numpy(), ref) < 2e-5
    # scaled up: extra free indices p0.. on A (after b) and q0.. on B (after h)
    P = list(range(100, 105))
    Q = list(range(200, 205))
    la2 = [a, b] + P + [c, d, e, f, g]
    lb2 = [h] + Q + [a, f, i]
    lc2 = [b, c] + P + [d, e, g, h] + Q + [i]
    x2 = rqcgen.random_complex(1 << len(la2), 56)
    y2 = rqcgen.random_complex(1 << len(lb2), 57)
    ref2 = oracle.einsum_step(x2, y2, la2, lb2, lc2)
    for kernel in (0, -1):
        got = R.pair_contract(_dev_c64(x2), _dev_c64(y2), la2, lb2, lc2, kernel=kernel)
        torch.cuda.synchronize()
        assert _rel_rms(got.cpu().numpy(), ref2) < 2e-5, kernel
