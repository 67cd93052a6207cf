"""Kernel-level parity of the 16-bit storage paths (Section 5.5: reduced
precision; half storage with FP32 arithmetic for memory-bound steps).

Operands are stored as packed (re, im) FP16 or BF16 pairs.  The reference
is numpy.einsum in complex128 on the operands' stored values (the 16-bit
values converted exactly), so:

* when every multiplied value is already 16-bit (both operands stored in
  16 bits), the products are exact in FP32 and only the FP32 accumulation
  rounds: error <= 2e-5 x RMS, on the 16-bit matrix cores as well as with
  FP32 arithmetic;
* when a complex64 operand meets the 16-bit matrix cores it is rounded to
  16 bits inside the kernel: error at the 16-bit level (FP16 u = 2^-11,
  BF16 u = 2^-8), bounded by 6e-3 / 4e-2 x RMS and above 1e-6 (the 16-bit
  products ran);
* a 16-bit output adds one rounding of the result at the same level.
"""
import sys

import numpy as np
import pytest

import rqcgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2110_14502_amd")

LP_TOL = {R.ST_F16: 6e-3, R.ST_BF16: 4e-2}
TORCH16 = {R.ST_F16: torch.float16, R.ST_BF16: torch.bfloat16}
MMA = {R.ST_F16: R.F16, R.ST_BF16: R.BF16}


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _store(x, st):
    """Device tensor of x in storage `st` and the complex128 values it holds."""
    t = torch.view_as_real(torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64))))
    if st != R.ST_C64:
        t = t.to(TORCH16[st])
    held = t.float().numpy()
    return t.contiguous().cuda(), held[..., 0].astype(np.float64) + 1j * held[..., 1]


def _empty(n, st):
    dt = torch.float32 if st == R.ST_C64 else TORCH16[st]
    return torch.empty((n, 2), dtype=dt, device="cuda")


def _values(t):
    h = t.float().cpu().numpy()
    return h[..., 0].astype(np.float64) + 1j * h[..., 1]


def _rel_rms(got, ref):
    return float(np.max(np.abs(got - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2)))


def _plan_layout(m, n, k, seed):
    """Summed labels lowest in both operands, same order (the planner's
    layouts); random orders elsewhere."""
    rng = np.random.default_rng(seed)
    M, N, K = list(range(m)), list(range(100, 100 + n)), list(range(200, 200 + k))
    la = [M[i] for i in rng.permutation(m)] + K
    lb = [N[i] for i in rng.permutation(n)] + K
    lc = M + N
    lc = [lc[i] for i in rng.permutation(len(lc))]
    return la, lb, lc


def _run(m, n, k, seed, sa, sb, sc, kernel, batch=1, mma=None, variant=0):
    la, lb, lc = _plan_layout(m, n, k, seed)
    a = rqcgen.random_complex((batch, 1 << (m + k)), seed)
    b = rqcgen.random_complex(1 << (n + k), seed + 1)
    A, a_held = _store(a.reshape(-1), sa)
    B, b_held = _store(b, sb)
    C = _empty(batch << (m + n), sc)
    if mma is None:
        mma = R.F32
    R.pair_contract_stored(A, B, C, la, lb, lc, sa, sb, sc, kernel, mma_prec=mma, batch=batch,
                           stride_a=1 << (m + k), stride_b=0, stride_c=1 << (m + n),
                           variant=variant)
    torch.cuda.synchronize()
    got = _values(C).reshape(batch, -1)
    a_held = a_held.reshape(batch, -1)
    errs = []
    for i in range(batch):
        ref = oracle.einsum_step(a_held[i], b_held, la, lb, lc)
        errs.append(_rel_rms(got[i], ref))
    return max(errs)


LP = [R.ST_F16, R.ST_BF16]


@pytest.mark.parametrize("lp", LP)
def test_rows_kernel_16bit_matrix_cores(lp):
    """Row-streaming kernel with A stored in 16 bits and sums of 16..256
    complex values: the 16-bit matrix-core path (16x16x32), in one chunk of
    16, then in one, two, four and eight chunks of 32."""
    for (m, n, k, seed) in ((13, 3, 4, 51), (12, 5, 5, 52), (11, 2, 6, 53), (10, 3, 7, 54),
                            (11, 4, 8, 55)):
        _say("rows 16-bit mma", lp, m, n, k)
        # both operands 16-bit: exact products, FP32 accumulation
        err = _run(m, n, k, seed, lp, lp, R.ST_C64, R.KERN_ROWS, batch=2)
        assert err < 2e-5, (m, n, k, err)
        # complex64 B rounded to 16 bits in the kernel
        err = _run(m, n, k, seed, lp, R.ST_C64, R.ST_C64, R.KERN_ROWS)
        assert 1e-6 < err < LP_TOL[lp], (m, n, k, err)
        # 16-bit output
        err = _run(m, n, k, seed, lp, lp, lp, R.KERN_ROWS)
        assert 1e-6 < err < LP_TOL[lp], (m, n, k, err)


@pytest.mark.parametrize("lp", LP)
def test_rows_kernel_wide_outputs_16bit(lp):
    """Row-streaming kernel on 64- and 128-column outputs with a 16-bit
    stored A: sums of 16 on the 16-bit matrix cores, shorter sums in FP32."""
    for (m, n, k, seed) in ((12, 7, 4, 131), (11, 6, 4, 132), (12, 7, 3, 133), (9, 6, 1, 134)):
        _say("rows wide 16-bit", lp, m, n, k)
        err = _run(m, n, k, seed, lp, lp, R.ST_C64, R.KERN_ROWS, batch=2)
        assert err < 2e-5, (m, n, k, err)
        err = _run(m, n, k, seed, lp, lp, lp, R.KERN_ROWS)
        assert 1e-6 < err < LP_TOL[lp], (m, n, k, err)


@pytest.mark.parametrize("lp", LP)
def test_rows_kernel_half_storage_fp32_arithmetic(lp):
    """Row-streaming kernel with short sums (k <= 3) on a 16-bit stored A:
    the values are converted and multiplied in FP32."""
    for (m, n, k, seed) in ((14, 3, 3, 61), (12, 2, 1, 62), (13, 4, 2, 63), (10, 0, 3, 64)):
        _say("rows half storage", lp, m, n, k)
        err = _run(m, n, k, seed, lp, R.ST_C64, R.ST_C64, R.KERN_ROWS, batch=2)
        assert err < 2e-5, (m, n, k, err)


@pytest.mark.parametrize("lp", LP)
def test_simt_kernel_half_storage_fp32_arithmetic(lp):
    """Generic kernel on 16-bit stored operands (FP32 arithmetic)."""
    cases = ((9, 4, 3, 71), (12, 6, 5, 72), (6, 6, 8, 73))
    for (m, n, k, seed) in cases:
        _say("simt half storage", lp, m, n, k)
        for sa, sb in ((lp, R.ST_C64), (R.ST_C64, lp), (lp, lp)):
            err = _run(m, n, k, seed, sa, sb, R.ST_C64, R.KERN_SIMT)
            assert err < 2e-5, (m, n, k, sa, sb, err)
        err = _run(m, n, k, seed, lp, lp, lp, R.KERN_SIMT)
        assert 1e-6 < err < LP_TOL[lp], (m, n, k, err)


@pytest.mark.parametrize("lp", LP)
def test_fp32_mfma_kernel_half_storage(lp):
    """FP32 matrix cores on 16-bit stored operands."""
    for (m, n, k, seed) in ((9, 7, 4, 81), (10, 6, 6, 82), (8, 8, 8, 83)):
        _say("mfma32 half storage", lp, m, n, k)
        err = _run(m, n, k, seed, lp, lp, R.ST_C64, R.KERN_MFMA, batch=2)
        assert err < 2e-5, (m, n, k, err)
        err = _run(m, n, k, seed, lp, R.ST_C64, lp, R.KERN_MFMA)
        assert 1e-6 < err < LP_TOL[lp], (m, n, k, err)


@pytest.mark.parametrize("lp", LP)
def test_16bit_mfma_kernel_stored_operands(lp):
    """16-bit matrix cores (32x32x16) on 16-bit stored operands: exact
    products, FP32 accumulation; and with complex64 operands rounded in
    the kernel."""
    for (m, n, k, seed) in ((9, 7, 4, 91), (10, 6, 5, 92), (8, 7, 8, 93)):
        _say("mfma16 stored", lp, m, n, k)
        err = _run(m, n, k, seed, lp, lp, R.ST_C64, R.KERN_MFMA16, batch=2, mma=MMA[lp])
        assert err < 2e-5, (m, n, k, err)
        err = _run(m, n, k, seed, R.ST_C64, R.ST_C64, R.ST_C64, R.KERN_MFMA16, mma=MMA[lp])
        assert 1e-6 < err < LP_TOL[lp], (m, n, k, err)
        err = _run(m, n, k, seed, lp, lp, lp, R.KERN_MFMA16, mma=MMA[lp])
        assert 1e-6 < err < LP_TOL[lp], (m, n, k, err)


def test_stored_entry_rejects_unsupported_requests():
    la, lb, lc = _plan_layout(6, 2, 2, 1)
    A, _ = _store(rqcgen.random_complex(1 << 8, 1), R.ST_C64)
    B, _ = _store(rqcgen.random_complex(1 << 4, 2), R.ST_C64)
    C = _empty(1 << 8, R.ST_C64)
    with pytest.raises(R.RqcError):   # too small for the FP32 matrix cores
        R.pair_contract_stored(A, B, C, la, lb, lc, 0, 0, 0, R.KERN_MFMA)
    with pytest.raises(R.RqcError):   # FP16 and BF16 in one call
        R.pair_contract_stored(A, B, C, la, lb, lc, R.ST_F16, R.ST_BF16, 0, R.KERN_SIMT)
    with pytest.raises(R.RqcError):   # 16-bit matrix cores need an MMA type
        R.pair_contract_stored(A, B, C, la, lb, lc, 0, 0, 0, R.KERN_MFMA16, mma_prec=R.F32)


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
def test_fp32_mfma_variants_vs_einsum(variant):
    """Every variant of the FP32 matrix-core kernel (three or four real
    products per complex product; per-tile or persistent walk) against
    einsum, on random index orders of A, B and C, short and long sums."""
    _say("mfma32 variant", variant)
    for (ra, rb, s, seed) in ((14, 12, 5, 3), (16, 13, 7, 4), (18, 16, 9, 8), (15, 15, 4, 5)):
        st = rqcgen.synthetic_step(ra, rb, s, seed)
        a = rqcgen.random_complex(1 << ra, seed + 100)
        b = rqcgen.random_complex(1 << rb, seed + 200)
        A, _ = _store(a, R.ST_C64)
        B, _ = _store(b, R.ST_C64)
        C = _empty(1 << len(st.labels_c), R.ST_C64)
        R.pair_contract_stored(A, B, C, st.labels_a, st.labels_b, st.labels_c, R.ST_C64,
                               R.ST_C64, R.ST_C64, R.KERN_MFMA, variant=variant)
        torch.cuda.synchronize()
        ref = oracle.einsum_step(a, b, st.labels_a, st.labels_b, st.labels_c)
        err = _rel_rms(_values(C), ref)
        assert err < 2e-5, (ra, rb, s, variant, err)
    # Sums of 16 over batches (the persistent walk crosses copies): fewer
    # items than workgroups, a little more than one round of them, and many.
    for (m, n, seed, batch) in ((7, 6, 21, 3), (10, 9, 22, 9), (12, 8, 23, 5)):
        err = _run(m, n, 4, seed, R.ST_C64, R.ST_C64, R.ST_C64, R.KERN_MFMA, batch=batch,
                   variant=variant)
        assert err < 2e-5, (m, n, batch, variant, err)


@pytest.mark.parametrize("variant", [R.VAR_SWAP, R.VAR_SWAP | R.VAR_TILES,
                                     R.VAR_SWAP | R.VAR_PERSISTENT, R.VAR_SWAP | R.VAR_4M,
                                     R.VAR_SWAP | R.VAR_PERSISTENT | R.VAR_4M])
def test_fp32_mfma_exchanged_operands_vs_einsum(variant):
    """The FP32 matrix-core kernel with A and B exchanged inside the kernel
    (B's free indices on the tile rows) against einsum: outputs of 128 and
    256 columns on random index orders, one and several K chunks, and a
    batch with a per-copy A and a shared B (strides exchanged with the
    operands)."""
    _say("mfma32 exchanged operands", variant)
    for (ra, rb, s, seed) in ((14, 12, 5, 13), (18, 15, 8, 14), (20, 16, 8, 15), (13, 11, 4, 16)):
        st = rqcgen.synthetic_step(ra, rb, s, seed)
        a = rqcgen.random_complex(1 << ra, seed + 100)
        b = rqcgen.random_complex(1 << rb, seed + 200)
        A, _ = _store(a, R.ST_C64)
        B, _ = _store(b, R.ST_C64)
        C = _empty(1 << len(st.labels_c), R.ST_C64)
        R.pair_contract_stored(A, B, C, st.labels_a, st.labels_b, st.labels_c, R.ST_C64,
                               R.ST_C64, R.ST_C64, R.KERN_MFMA, variant=variant)
        torch.cuda.synchronize()
        ref = oracle.einsum_step(a, b, st.labels_a, st.labels_b, st.labels_c)
        err = _rel_rms(_values(C), ref)
        assert err < 2e-5, (ra, rb, s, variant, err)
    err = _run(9, 7, 5, 17, R.ST_C64, R.ST_C64, R.ST_C64, R.KERN_MFMA, batch=3, variant=variant)
    assert err < 2e-5, err
    # B's free indices must fill a row tile: seven or more.
    la, lb, lc = _plan_layout(10, 6, 4, 18)
    A, _ = _store(rqcgen.random_complex(1 << 14, 1), R.ST_C64)
    B, _ = _store(rqcgen.random_complex(1 << 10, 2), R.ST_C64)
    C = _empty(1 << 16, R.ST_C64)
    with pytest.raises(R.RqcError):
        R.pair_contract_stored(A, B, C, la, lb, lc, 0, 0, 0, R.KERN_MFMA, variant=variant)


@pytest.mark.parametrize("lp", LP)
def test_16bit_mfma_exchanged_operands(lp):
    """The 16-bit matrix-core kernel with A and B exchanged inside the
    kernel (B's free indices on the tile rows) against einsum on the stored
    values: outputs of 128 and 256 columns, sums of 16..128 terms, batched
    copies with a per-copy A and a shared B, both operands in 16 bits (exact
    products) and B in complex64 (converted for the matrix cores)."""
    for (m, n, k, seed) in ((10, 7, 4, 111), (12, 7, 5, 112), (9, 8, 6, 113), (11, 7, 7, 114)):
        _say("mfma16 exchanged operands", lp, m, n, k)
        err = _run(m, n, k, seed, lp, lp, R.ST_C64, R.KERN_MFMA16, batch=3, mma=MMA[lp],
                   variant=R.VAR_SWAP)
        assert err < 2e-5, (m, n, k, err)
        err = _run(m, n, k, seed, lp, R.ST_C64, lp, R.KERN_MFMA16, batch=2, mma=MMA[lp],
                   variant=R.VAR_SWAP)
        assert 1e-6 < err < LP_TOL[lp], (m, n, k, err)
    # B's free indices must fill a row tile: seven or more.
    la, lb, lc = _plan_layout(10, 6, 5, 115)
    A, _ = _store(rqcgen.random_complex(1 << 15, 1), lp)
    B, _ = _store(rqcgen.random_complex(1 << 11, 2), lp)
    C = _empty(1 << 16, R.ST_C64)
    with pytest.raises(R.RqcError):
        R.pair_contract_stored(A, B, C, la, lb, lc, lp, lp, 0, R.KERN_MFMA16, mma_prec=MMA[lp],
                               variant=R.VAR_SWAP)


@pytest.mark.parametrize("lp", LP)
def test_16bit_mfma_streaming_variant(lp):
    """The 16-bit matrix-core kernel's streaming form (A streamed past a
    resident tile of B over the whole sum), sums of 32..128 terms, several
    row and column tiles, batched copies, against einsum on the stored
    values."""
    for (m, n, k, seed) in ((10, 7, 5, 101), (9, 6, 6, 102), (11, 7, 7, 103), (8, 8, 7, 104)):
        _say("mfma16 stream", lp, m, n, k)
        err = _run(m, n, k, seed, lp, lp, R.ST_C64, R.KERN_MFMA16, batch=3, mma=MMA[lp],
                   variant=R.VAR_STREAM)
        assert err < 2e-5, (m, n, k, err)
        err = _run(m, n, k, seed, lp, R.ST_C64, lp, R.KERN_MFMA16, batch=2, mma=MMA[lp],
                   variant=R.VAR_STREAM)
        assert 1e-6 < err < LP_TOL[lp], (m, n, k, err)
