"""A slice share of a 10x10 (1+20+1) circuit: 256 slices (eight enumerated
sliced wires, every other sliced wire fixed to 0, single-valued wires
pruned) under a 2^24 per-slice bound, all 256 in one call per precision.
(The benchmark runs the 1024-slice share at 2^28; this size keeps the
oracle's work to seconds per slice.)

The oracle's own greedy order does not fit in memory on this network, so it
contracts its own gate tensors in the plan's order given as data (the order
changes cost, never the value).  Checked:
* 4 of the slices against the oracle;
* 32 checked slices, FP16 and BF16 against FP32 within the reduced-precision
  tolerance;
* sub-slices of the 32 checked slices (up to 40 more wires fixed, half of
  them drawn at random) against the oracle.
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

ROWS, COLS, DEPTH, SEED, BOUND, LOCAL, TRIALS = 10, 10, 20, 4, 24, 8, 64
N = ROWS * COLS


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def share():
    _say("share plan + FP32 over 256 slices")
    circ = rqcgen.grid_rqc(ROWS, COLS, DEPTH, SEED)
    bits = rqcgen.random_bits(N, SEED)
    net = R.Network(R.Circuit.from_rqcgen(circ), [])
    plan = R.Plan(net, max_log2_elems=BOUND, path_trials=TRIALS, seed=SEED,
                  n_local_sliced=LOCAL).bind()
    free, _ = torch.cuda.mem_get_info()
    ws = torch.empty(int(min(free * 0.6, 160 << 30)), dtype=torch.uint8, device="cuda")
    _, per = plan.contract(bits, per_slice=True, workspace=ws)
    per32 = R.to_complex(per)[:, 0, 0]
    checked = sorted(int(x) for x in np.random.default_rng(SEED).choice(1 << LOCAL, 32, replace=False))
    yield circ, bits, net, plan, ws, per32, checked
    del ws


def _wires(plan):
    return plan.sliced_wires(), [w[:2] for w in plan.fixed_wires()]


def _err(got, ref, plan):
    """Per-slice error over the checked slices, in units of the larger of
    their RMS and the natural scale of one slice, 2^-(n+S)/2 (S sliced wires
    in all: 2^S slices of random phase summing to an amplitude of RMS size
    2^-n/2).  Some slices cancel to values many orders below that scale,
    where FP32 returns its rounding noise; that noise is negligible at the
    natural scale, and measured against it."""
    n_sliced = len(plan.sliced_wires()) + len(plan.fixed_wires())
    natural = 2.0 ** (-(N + n_sliced) / 2)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2))
    return np.max(np.abs(got - ref)) / max(rms, natural)


def test_share_values_are_finite_and_not_all_zero(share):
    _, _, _, plan, _, per32, checked = share
    assert np.all(np.isfinite(per32))
    assert np.count_nonzero(per32) > 0
    assert plan.last_report["fp32_reruns"] == 0


def test_share_slices_vs_oracle(share):
    circ, bits, _, plan, _, per32, checked = share
    _say("share slices vs oracle")
    e = plan.export()
    groups, pairs = oracle_order(circ, [], e)
    ids = checked[:4]
    ow, oids = oracle_wires_and_ids(e, ids)
    ref = oracle.slice_values_ordered(circ, [], bits, ow, oids, groups, pairs)[:, 0]
    assert _err(per32[ids], ref, plan) < 1e-4


# FP16 meets the reduced-precision bound per slice.  BF16 keeps 8
# significand bits: on these slices, whose values are far smaller than the
# terms that cancel to form them, its per-slice error measured 0.02-0.05;
# the bound states that, and the fidelity bound is the same for both.
@pytest.mark.parametrize("prec,tol", [("f16", 2e-2), ("bf16", 6e-2)])
def test_share_reduced_precision_vs_fp32(share, prec, tol):
    _, bits, _, plan, ws, per32, checked = share
    _say("share", prec)
    _, per = plan.contract(bits, per_slice=True, prec=R.PRECISIONS[prec], workspace=ws)
    lp = R.to_complex(per)[:, 0, 0]
    assert np.all(np.isfinite(lp))
    assert _err(lp[checked], per32[checked], plan) < tol
    if np.sqrt(np.mean(np.abs(per32[checked]) ** 2)) > 2.0 ** (-(N + len(plan.sliced_wires()) + len(plan.fixed_wires())) / 2):
        assert oracle.linear_fidelity(lp[checked], per32[checked]) > 0.99


def test_share_subslices_vs_oracle(share):
    circ, bits, net, plan, ws, _, checked = share
    _say("share sub-slices vs oracle")
    loc, fixed = _wires(plan)
    q = R.Plan(net, max_log2_elems=21, path_trials=16, seed=SEED, forced_wires=loc + fixed,
               n_local_sliced=LOCAL)
    extra = [w[:2] for w in q.fixed_wires()[len(fixed):]]
    x = min(40, len(extra))
    wires = loc + extra[:x] + fixed + extra[x:]
    fine = R.Plan(net, n_sliced=len(wires), forced_wires=wires, path_trials=16, seed=SEED,
                  n_local_sliced=LOCAL + x).bind()
    assert fine.sliced_wires() == loc + extra[:x]
    rng = np.random.default_rng(7)
    # Half of the sub-slices keep the extra wires at 0, half draw them.
    ids = [s + ((int(rng.integers(1 << x)) if i % 2 else 0) << LOCAL) for i, s in enumerate(checked)]
    _, per = fine.contract(bits, slice_ids=ids, per_slice=True, workspace=ws)
    got = R.to_complex(per)[:, 0, 0]
    e = fine.export()
    groups, pairs = oracle_order(circ, [], e)
    ow, oids = oracle_wires_and_ids(e, ids)
    assert ow[:len(wires)] == wires
    ref = oracle.slice_values_ordered(circ, [], bits, ow, oids, groups, pairs)[:, 0]
    assert _err(got, ref, fine) < 1e-4


def test_share_slices_equal_full_plan_slices():
    """A share with high bits b computes slices b*2^L + i of the full
    slicing: checked against the full plan and the oracle on a 5x5 circuit."""
    _say("share vs full plan")
    c = rqcgen.grid_rqc(5, 5, 8, 2)
    openq = [23, 24]
    net = R.Network(R.Circuit.from_rqcgen(c), openq)
    bits = rqcgen.random_bits(23, 3)
    full = R.Plan(net, n_sliced=8, path_trials=32, seed=1).bind()
    wires = full.sliced_wires()
    _, per_full = full.contract(bits, per_slice=True)
    per_full = R.to_complex(per_full)[:, 0]
    for high in ([1, 0, 1], [0, 1, 1]):
        share = R.Plan(net, n_sliced=8, forced_wires=wires, path_trials=32, seed=5,
                       n_local_sliced=5, share_bits=high).bind()
        _, per = share.contract(bits, per_slice=True)
        per = R.to_complex(per)[:, 0]
        base = sum(b << i for i, b in enumerate(high)) << 5
        ref = per_full[base:base + 32]
        assert np.max(np.abs(per - ref)) * 2 ** 12.5 < 1e-4
    ids = [base + 3, base + 17]
    o = oracle.slice_values_tn(c, openq, bits, wires, ids)
    assert np.max(np.abs(per_full[ids] - o)) * 2 ** 12.5 < 1e-4


def test_group_limit_does_not_change_results():
    _say("group limit")
    c = rqcgen.grid_rqc(5, 5, 10, 4)
    openq = [20, 21, 22, 23, 24]
    net = R.Network(R.Circuit.from_rqcgen(c), openq)
    bits = rqcgen.random_bits(20, 1)
    p = R.Plan(net, n_sliced=6, path_trials=32, seed=3).bind()
    ref = R.to_complex(p.contract(bits))[0]
    for g in (1, 3, 16):
        p.set_group_limit(g)
        got = R.to_complex(p.contract(bits))[0]
        assert p.last_report["slices_per_group"] <= g
        assert np.max(np.abs(got - ref)) * 2 ** 12.5 < 1e-5
    p.set_group_limit(0)
    assert oracle.normalized_error(ref, oracle.amplitudes_tn(c, openq, bits), 25) < 1e-4
