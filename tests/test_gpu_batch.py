"""A large correlated batch (Appendix A: fix some qubits, exhaust the rest,
score the bunch by the linear cross-entropy benchmark) and its statistics.

The 6x6 (1+12+1) circuit with 21 open qubits: 2^21 amplitudes from one
sliced contraction.  Checked against the oracle on the 64 entries whose
qubits 15..29 take a seeded pattern (stored oracle values,
tests/golden/batch6_amplitudes.txt), and the device statistics (sums,
linear cross-entropy) against the oracle's formulas on the copied batch.
"""
import sys

import numpy as np
import pytest

import rqcgen
import oracle
from golden_io import read_golden

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
R = pytest.importorskip("paper_2110_14502_amd")

N, N_OPEN = 36, 21
OPEN = list(range(N - N_OPEN, N))


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def batch():
    _say("batch 2^21 plan + fp32")
    c = rqcgen.grid_rqc(6, 6, 12, 2)
    bits = rqcgen.random_bits(15, 3)
    P = R.Plan(R.Network(R.Circuit.from_rqcgen(c), OPEN), max_log2_elems=28, path_trials=128,
               seed=1).bind()
    out = P.contract(bits).clone()
    pattern = rqcgen.random_bits(15, 4)
    base = sum(int(b) << i for i, b in enumerate(pattern))
    entries = base + (np.arange(64, dtype=np.int64) << 15)
    return c, bits, P, out, entries


def test_batch_subset_vs_oracle(batch):
    _, _, P, out, entries = batch
    assert out.numel() == 2 << N_OPEN
    got = R.to_complex(out)[0][entries]
    idx, ref = read_golden("batch6_amplitudes.txt")
    assert list(idx) == list(range(64))
    assert oracle.normalized_error(got, ref, N) < 1e-4
    assert oracle.linear_fidelity(got, ref) > 0.999999


def test_batch_statistics_on_device(batch):
    _, _, _, out, entries = batch
    _say("batch statistics")
    host = R.to_complex(out)[0]
    samples = torch.from_numpy(entries).cuda()
    st = R.batch_xeb(out, N, samples=samples)
    p = np.abs(host) ** 2
    assert abs(st["sum_p"] / p.sum() - 1) < 1e-12
    assert abs(st["sum_p2"] / np.sum(p * p) - 1) < 1e-12
    assert abs(st["xeb_all"] - (2.0 ** N * p.mean() - 1)) < 1e-9
    assert abs(st["xeb_ideal_sampling"] - oracle.xeb_ideal_sampling(host, N)) < 1e-9
    assert abs(st["xeb_samples"] - oracle.xeb_of_samples(host, N, entries)) < 1e-9
    # Porter-Thomas within the bunch: ideal sampling scores about 1.
    assert 0.8 < st["xeb_ideal_sampling"] < 1.2
    # an index outside the batch is reported as NaN, not read
    bad = torch.tensor([0, 1 << N_OPEN], dtype=torch.int64, device="cuda")
    assert np.isnan(R.batch_xeb(out, N, samples=bad)["xeb_samples"])


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_batch_reduced_precision(batch, prec):
    _, bits, P, out, entries = batch
    _say("batch", prec)
    lp = P.contract(bits, prec=R.PRECISIONS[prec])
    got = R.to_complex(lp)[0]
    _, ref = read_golden("batch6_amplitudes.txt")
    err = oracle.normalized_error(got[entries], ref, N)
    assert 1e-6 < err < 2e-2, err
    f32 = R.to_complex(out)[0]
    assert oracle.linear_fidelity(got, f32) > 0.99
    st = R.batch_xeb(lp, N)
    assert abs(st["xeb_ideal_sampling"] - oracle.xeb_ideal_sampling(f32, N)) < 2e-2
