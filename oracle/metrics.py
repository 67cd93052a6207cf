"""Error measures.  The paper gives no error metric beyond "within 1%"
(Section 5.5) and a Porter-Thomas comparison (Section 6.2); the measures
used are:

* normalised error: max |a - a_ref| * 2^(n/2), i.e. relative to the RMS
  amplitude 2^(-n/2) of an n-qubit state;
* linear fidelity: |<a_ref, a>|^2 / (<a_ref, a_ref> <a, a>);
* per-slice error: max |s - s_ref| / RMS(s_ref) over the checked slices;
* slice error at the natural scale: max |s - s_ref| divided by the larger of
  RMS(s_ref) and the natural size of one slice, 2^(-(n+S)/2) for S sliced
  wires in all (2^S slices of random phase add up to an amplitude of RMS
  size 2^(-n/2)).  Some slice sets cancel to values far below that scale;
  measured against their own RMS, any rounding would look large there.
"""
import numpy as np


def normalized_error(a, ref, n_qubits):
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    ref = np.asarray(ref, dtype=np.complex128).reshape(-1)
    return float(np.max(np.abs(a - ref)) * 2.0 ** (n_qubits / 2.0))


def linear_fidelity(a, ref):
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    ref = np.asarray(ref, dtype=np.complex128).reshape(-1)
    num = abs(np.vdot(ref, a)) ** 2
    den = np.vdot(ref, ref).real * np.vdot(a, a).real
    return float(num / den) if den > 0 else 0.0


def per_slice_error(s, ref):
    s = np.asarray(s, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    return float(np.max(np.abs(s - ref)) / rms) if rms > 0 else float(np.max(np.abs(s)))


def natural_slice_scale(n_qubits, n_sliced_total):
    """RMS size of one slice of an n-qubit amplitude cut on S wires."""
    return 2.0 ** (-(n_qubits + n_sliced_total) / 2.0)


def slice_error_natural(s, ref, n_qubits, n_sliced_total):
    s = np.asarray(s, dtype=np.complex128).reshape(-1)
    ref = np.asarray(ref, dtype=np.complex128).reshape(-1)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    scale = max(rms, natural_slice_scale(n_qubits, n_sliced_total))
    return float(np.max(np.abs(s - ref)) / scale)


def xeb_of_samples(amps, n_qubits, samples):
    """Linear cross-entropy benchmark (the XEB of Section 2 and Appendix A)
    of the bitstrings `samples` (indices into the amplitude batch `amps`):
    2^n times the mean ideal probability |a|^2 of the samples, minus 1."""
    amps = np.asarray(amps, dtype=np.complex128).reshape(-1)
    p = np.abs(amps[np.asarray(samples, dtype=np.int64)]) ** 2
    return float(2.0 ** n_qubits * np.mean(p) - 1.0)


def xeb_ideal_sampling(amps, n_qubits):
    """The expected linear cross-entropy of bitstrings drawn from the batch
    with probability proportional to |a|^2 (perfect sampling restricted to
    the batch): 2^n * sum |a|^4 / sum |a|^2 - 1."""
    p = np.abs(np.asarray(amps, dtype=np.complex128).reshape(-1)) ** 2
    return float(2.0 ** n_qubits * np.sum(p * p) / np.sum(p) - 1.0)
