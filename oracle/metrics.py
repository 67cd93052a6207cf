"""Error measures.  The paper gives no error metric beyond "within 1%"
(Section 5.5) and a Porter-Thomas comparison (Section 6.2); the measures
used are:

* normalised error: max |a - a_ref| * 2^(n/2), i.e. relative to the RMS
  amplitude 2^(-n/2) of an n-qubit state;
* linear fidelity: |<a_ref, a>|^2 / (<a_ref, a_ref> <a, a>);
* per-slice error: max |s - s_ref| / RMS(s_ref) over the checked slices.
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
