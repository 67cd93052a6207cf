"""CPU oracle for sliced tensor-network amplitudes of random quantum circuits.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
native library (no gate tables, no layout helpers, no generators beyond the
seeded input module ``rqcgen``), and it never takes an expected value from
the GPU path.

Everything is plain numpy in complex128:

* ``gates``       -- gate matrices written from their textbook definitions;
* ``statevector`` -- brute-force Schroedinger simulation (Section 3.2, first
  class of simulators), used as the ground truth for small circuits;
* ``tn``          -- one tensor per gate (Section 3.2, tensor approach),
  optional slicing of wires (Section 5.1), pairwise contraction with
  ``numpy.tensordot`` in a plain greedy order, or in an order given as
  data (``contract_ordered``: the order changes cost, never the value);
* ``step``        -- a single pairwise contraction (Section 5.4) by
  ``numpy.einsum``, and by direct summation at sampled output coordinates;
* ``metrics``     -- normalised error, linear fidelity, per-slice errors.

Pins (see ``tests/test_oracle_pins.py``) tie each function to something
other than itself: state vector vs tensor network, unitarity, the slice sum
against the unsliced contraction, mirror circuits, product states in closed
form, textbook gate identities, Porter-Thomas statistics and brute force on
tiny inputs.
"""
from .gates import gate_matrix, H_M, SQRT_X_M, SQRT_Y_M, SQRT_W_M, fsim
from .statevector import statevector, amplitudes_sv, bit_index
from .tn import (build_network, contract_network, amplitudes_tn,
                 slice_values_tn, wire_labels, contract_ordered, slice_values_ordered)
from .step import einsum_step, sampled_step
from .metrics import (normalized_error, linear_fidelity, per_slice_error,
                      natural_slice_scale, slice_error_natural, xeb_of_samples,
                      xeb_ideal_sampling)

__all__ = [
    "gate_matrix", "H_M", "SQRT_X_M", "SQRT_Y_M", "SQRT_W_M", "fsim",
    "statevector", "amplitudes_sv", "bit_index",
    "build_network", "contract_network", "amplitudes_tn", "slice_values_tn",
    "contract_ordered", "slice_values_ordered",
    "wire_labels", "einsum_step", "sampled_step",
    "normalized_error", "linear_fidelity", "per_slice_error",
    "natural_slice_scale", "slice_error_natural", "xeb_of_samples", "xeb_ideal_sampling",
]
