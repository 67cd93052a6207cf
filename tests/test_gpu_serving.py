"""Serving loop (continuous batching) on the GPU: results alone vs in a mix,
against the oracle, plan reuse, batching, and admission by device budget."""
import sys
import time

import numpy as np
import pytest

import rqcgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2110_14502_amd")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _requests():
    """Mixed sizes, open counts and precisions; some share circuits."""
    reqs = []
    specs = [(4, 4, 8, 1, 4, R.F32), (5, 5, 8, 2, 2, R.F32), (4, 5, 10, 3, 0, R.F16),
             (5, 5, 10, 4, 6, R.F32), (4, 4, 8, 1, 4, R.F32), (5, 5, 8, 2, 3, R.F16),
             (3, 4, 6, 5, 8, R.F32), (5, 5, 10, 4, 6, R.F32)]
    for i, (r, c, d, seed, n_open, prec) in enumerate(specs):
        circ = rqcgen.grid_rqc(r, c, d, seed)
        n = r * c
        openq = list(range(n - n_open, n))
        bits = rqcgen.random_bits(n - n_open, 100 + i)
        reqs.append((circ, openq, bits, prec))
    return reqs


def _collect(srv, tickets, timeout=120):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for r in srv.poll():
            out[r["ticket"]] = r
        if time.time() - t0 > timeout:
            raise TimeoutError("server did not finish")
        time.sleep(0.002)
    return [out[t] for t in tickets]


def _submit(srv, req):
    circ, openq, bits, prec = req
    return srv.submit(circ.n_qubits, circ.gates, openq, bits, prec=prec, max_log2_elems=20)


def test_alone_vs_mix_and_vs_oracle():
    _say("serving alone vs mix")
    reqs = _requests()
    srv = R.Server(4 << 30, max_inflight=4, n_streams=4, max_batch=8)
    alone = []
    for q in reqs:
        t = _submit(srv, q)
        alone.append(_collect(srv, [t])[0])
    tickets = [_submit(srv, q) for q in reqs]
    mix = _collect(srv, tickets)
    st = srv.stats()
    srv.close()
    for q, a, m in zip(reqs, alone, mix):
        circ, openq, bits, prec = q
        assert a["status"] == 0 and m["status"] == 0
        n = circ.n_qubits
        # the same request gives the same amplitudes alone and in the mix
        assert np.max(np.abs(a["amplitudes"] - m["amplitudes"])) * 2 ** (n / 2) < 1e-9
        ref = oracle.amplitudes_tn(circ, openq, bits)
        tol = 1e-4 if prec == R.F32 else 2e-2
        assert oracle.normalized_error(m["amplitudes"], ref, n) < tol
        assert m["t_submit"] <= m["t_start"] <= m["t_done"]
    assert st["completed"] == 2 * len(reqs)
    assert st["plans_reused"] > 0
    assert st["max_inflight_seen"] >= 2


def test_admission_by_budget():
    _say("serving admission")
    circ = rqcgen.grid_rqc(5, 5, 10, 7)
    openq = list(range(19, 25))
    # A budget far below what the plan needs: the request fails with EHBM.
    tiny = R.Server(1 << 16, max_inflight=2)
    t = tiny.submit(25, circ.gates, openq, rqcgen.random_bits(19, 1), max_log2_elems=20)
    r = _collect(tiny, [t])[0]
    tiny.close()
    assert r["status"] == R.EHBM
    # A budget that holds about one call at a time still serves every request.
    P = R.Plan(R.Network(R.Circuit.from_rqcgen(circ), openq), max_log2_elems=20, path_trials=64)
    need = P.resident_bytes() + P.workspace_bytes(0, 1, R.F32)[0] + (1 << 20)
    srv = R.Server(int(need * 1.6), max_inflight=8, max_batch=1)
    tickets = [srv.submit(25, circ.gates, openq, rqcgen.random_bits(19, s), max_log2_elems=20)
               for s in range(6)]
    res = _collect(srv, tickets)
    st = srv.stats()
    srv.close()
    assert all(x["status"] == 0 for x in res)
    assert st["peak_bytes"] <= int(need * 1.6)
