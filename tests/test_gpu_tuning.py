"""Per-step kernel tuning, the precision pre-analysis and the half-storage
policy, each checked against the oracle.

* rqc_plan_autotune: every choice it can make gives the same amplitudes
  within FP32 rounding (and the oracle's within 1e-4); a second plan reads
  the same choices from the cache file without timing anything.
* rqc_plan_calibrate (Section 5.5 pre-analysis): on a plan that stores
  every intermediate from 2^6 elements in BF16 (per-slice error 2.3e-2 in
  that assignment), the sensitivity-driven assignment meets its target on
  the calibration slice and brings every slice within 2e-2 of the oracle.
* RQC_POLICY_STORAGE (half storage, FP32 arithmetic): 16-bit storage, no
  16-bit matrix-core step, error at the storage-rounding level.
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

N = 25
OPEN = [21, 22, 23, 24]


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _plan(**kw):
    c = rqcgen.grid_rqc(5, 5, 12, 3)
    return c, R.Plan(R.Network(R.Circuit.from_rqcgen(c), OPEN), n_sliced=4, seed=5,
                     path_trials=64, **kw).bind()


@pytest.fixture(scope="module")
def ref():
    c, P = _plan()
    bits = rqcgen.random_bits(21, 9)
    e = P.export()
    groups, pairs = oracle_order(c, OPEN, e)
    ow, oids = oracle_wires_and_ids(e, range(16))
    return bits, oracle.slice_values_ordered(c, OPEN, bits, ow, oids, groups, pairs)


def test_autotune_results_and_cache(ref, tmp_path):
    bits, slices = ref
    _say("autotune")
    _, P = _plan()
    before = R.to_complex(P.contract(bits))[0]
    cache = str(tmp_path / "tune.txt")
    rep = P.autotune(R.F32, cache_path=cache)
    assert rep["steps"] > 0 and rep["timed"] == rep["steps"] and rep["cached"] == 0
    assert rep["ms_tuned"] <= rep["ms_default"] * 1.0001
    after, per = P.contract(bits, per_slice=True)
    after = R.to_complex(after)[0]
    assert oracle.normalized_error(after, slices.sum(0), N) < 1e-4
    assert oracle.slice_error_natural(R.to_complex(per)[:, 0], slices, N, 4) < 1e-4
    assert oracle.normalized_error(after, before, N) < 1e-5
    kernels = [s["kernel"] for s in P.steps()]
    # a second plan of the same network reads every choice from the cache
    _, Q = _plan()
    rep2 = Q.autotune(R.F32, cache_path=cache)
    assert rep2["timed"] == 0 and rep2["cached"] == rep["steps"]
    assert [s["kernel"] for s in Q.steps()] == kernels
    got = R.to_complex(Q.contract(bits))[0]
    assert np.array_equal(got, after)
    # reduced precision is tuned on its own (its 16-bit matrix-core steps
    # have a choice only where the row kernel also applies)
    rep16 = P.autotune(R.F16)
    assert rep16["timed"] == rep16["steps"]
    lp = R.to_complex(P.contract(bits, prec=R.F16))[0]
    assert oracle.normalized_error(lp, slices.sum(0), N) < 2e-2


def test_calibration_brings_bf16_within_bound(ref):
    bits, slices = ref
    _say("calibrate bf16")
    _, P = _plan(lp_min_log2=6, bf16_min_log2=6, precision_policy=R.POLICY_CALIBRATED)
    _, per0 = P.contract(bits, prec=R.BF16, per_slice=True)
    err0 = oracle.slice_error_natural(R.to_complex(per0)[:, 0], slices, N, 4)
    n16_before = sum(s["lp_output_bf16"] for s in P.steps())
    rep = P.calibrate(bits, prec=R.BF16, slice_id=0, target_err=3e-3)
    assert rep["candidates"] > 0 and 0 < rep["reduced"] < rep["candidates"]
    assert rep["measured_err"] <= 3e-3
    assert rep["max_step_err"] > rep["min_step_err"]
    n16_after = sum(s["lp_output_bf16"] for s in P.steps())
    assert 0 < n16_after < n16_before
    amps, per = P.contract(bits, prec=R.BF16, per_slice=True)
    amps, per = R.to_complex(amps)[0], R.to_complex(per)[:, 0]
    err = oracle.slice_error_natural(per, slices, N, 4)
    assert 1e-6 < err < 2e-2 and err < err0, (err, err0)
    assert oracle.linear_fidelity(per, slices) > 0.99
    assert oracle.normalized_error(amps, slices.sum(0), N) < 2e-2
    # FP32 calls are unaffected
    a32 = R.to_complex(P.contract(bits))[0]
    assert oracle.normalized_error(a32, slices.sum(0), N) < 1e-4


def test_storage_policy_half_storage_fp32_arithmetic(ref):
    bits, slices = ref
    _say("storage policy")
    _, P = _plan(lp_min_log2=6, precision_policy=R.POLICY_STORAGE)
    steps = [s for s in P.steps() if s["depends_on_slice"]]
    assert sum(s["lp_output"] for s in steps) >= 10
    assert all(s["kernel_lp"] != R.KERN_MFMA16 for s in steps)
    amps = R.to_complex(P.contract(bits, prec=R.F16))[0]
    err = oracle.normalized_error(amps, slices.sum(0), N)
    assert 1e-6 < err < 2e-2, err
    assert oracle.linear_fidelity(amps, slices.sum(0)) > 0.999
