"""Slice shares on the host (no GPU): option checks, the exported fixed
wires, and the plan's tree used as the oracle's contraction order (the
oracle then checks its own greedy values and the state vector)."""
import numpy as np
import pytest

import rqcgen
import oracle
from plan_order import oracle_order, oracle_wires_and_ids

R = pytest.importorskip("paper_2110_14502_amd")


def _net(rows, cols, depth, seed, n_open):
    c = rqcgen.grid_rqc(rows, cols, depth, seed)
    n = rows * cols
    openq = list(range(n - n_open, n))
    return c, openq, R.Network(R.Circuit.from_rqcgen(c), openq)


def test_share_options_are_checked():
    _, _, net = _net(4, 4, 8, 1, 2)
    with pytest.raises(R.RqcError) as e:
        R.Plan(net, n_sliced=4, n_local_sliced=63)
    assert e.value.code == R.EINVAL
    with pytest.raises(R.RqcError) as e:
        R.Plan(net, n_sliced=4, n_local_sliced=5)
    assert e.value.code == R.EINVAL
    with pytest.raises(R.RqcError) as e:
        R.Plan(net, n_sliced=4, n_local_sliced=2, share_bits=[0, 2])
    assert e.value.code == R.EINVAL
    with pytest.raises(R.RqcError) as e:
        R.Plan(net, n_sliced=70, path_trials=4)
    assert e.value.code == R.EUNSUPPORTED


def test_wide_network_needs_a_share():
    """10x10 (1+20+1) under a 2^30 bound needs far more than 62 sliced
    wires: refused without a share, planned with one."""
    _, _, net = _net(10, 10, 20, 4, 0)
    with pytest.raises(R.RqcError) as e:
        R.Plan(net, max_log2_elems=30, path_trials=8, seed=4)
    assert e.value.code == R.EUNSUPPORTED
    p = R.Plan(net, max_log2_elems=30, path_trials=8, seed=4, n_local_sliced=10)
    info = p.info()
    assert info["n_slices"] == 1024 and info["max_log2_elems"] <= 30
    assert len(p.fixed_wires()) > 52
    assert all(v == 0 for _, _, v in p.fixed_wires())


def test_fixed_wires_follow_the_share_bits():
    c, openq, net = _net(5, 5, 8, 2, 2)
    full = R.Plan(net, n_sliced=8, path_trials=32, seed=1)
    wires = full.sliced_wires()
    share = R.Plan(net, n_sliced=8, forced_wires=wires, path_trials=32, seed=1,
                   n_local_sliced=5, share_bits=[1, 0, 1])
    assert share.info()["n_slices"] == 32
    assert share.sliced_wires() == wires[:5]
    assert share.fixed_wires() == [w + (v,) for w, v in zip(wires[5:], (1, 0, 1))]
    # Leaves carrying only fixed wires no longer depend on the slice.
    assert share.info()["n_invariant_steps"] >= full.info()["n_invariant_steps"]


def test_plan_tree_as_oracle_order_matches_statevector():
    c, openq, net = _net(4, 4, 8, 1, 4)
    p = R.Plan(net, path_trials=16, seed=3)
    closed = rqcgen.random_bits(12, 5)
    groups, pairs = oracle_order(c, openq, p.export())
    tensors, out = oracle.build_network(c, openq, closed)
    got = oracle.contract_ordered(tensors, out, groups, pairs)
    ref = oracle.amplitudes_sv(c, openq, closed)
    assert np.max(np.abs(got - ref)) * 2 ** 8 < 1e-12


def test_share_tree_as_oracle_order_matches_greedy_slices():
    c, openq, net = _net(4, 5, 8, 6, 1)
    p0 = R.Plan(net, n_sliced=7, path_trials=16, seed=2)
    wires = p0.sliced_wires()
    bits = [0, 1, 1, 0]
    share = R.Plan(net, n_sliced=7, forced_wires=wires, path_trials=16, seed=2,
                   n_local_sliced=3, share_bits=bits)
    closed = rqcgen.random_bits(19, 8)
    e = share.export()
    groups, pairs = oracle_order(c, openq, e)
    high = sum(b << i for i, b in enumerate(bits))
    ids = [i + (high << 3) for i in range(8)]
    ow, oids = oracle_wires_and_ids(e, range(8))
    got = oracle.slice_values_ordered(c, openq, closed, ow, oids, groups, pairs)
    ref = oracle.slice_values_tn(c, openq, closed, wires, ids)
    assert np.max(np.abs(got - ref)) * 2 ** 10 < 1e-12


def test_pruned_wires_carry_a_single_value():
    """The planner projects out wires whose leaf slab is zero at one value;
    the oracle confirms that fixing them to that value keeps the amplitude
    and that the other value gives zero."""
    c, openq, net = _net(5, 5, 10, 3, 2)
    p = R.Plan(net, path_trials=8, seed=1)
    pruned = p.pruned_wires()
    assert len(pruned) > 0
    closed = rqcgen.random_bits(23, 9)
    full = oracle.amplitudes_tn(c, openq, closed)
    wires = [w[:2] for w in pruned]
    ids = sum(v << i for i, (_, _, v) in enumerate(pruned))
    kept = oracle.slice_values_tn(c, openq, closed, wires, [ids])[0]
    assert np.max(np.abs(kept - full)) * 2 ** 12.5 < 1e-12
    for j in (0, len(pruned) - 1):
        flipped = oracle.slice_values_tn(c, openq, closed, wires, [ids ^ (1 << j)])[0]
        assert np.max(np.abs(flipped)) * 2 ** 12.5 < 1e-12
    # Forced wires are never pruned.
    q = R.Plan(net, n_sliced=1, forced_wires=[wires[0]], path_trials=8, seed=1)
    assert q.sliced_wires() == [wires[0]]
    assert wires[0] not in [w[:2] for w in q.pruned_wires()]
