"""Gate matrices in complex128, written from their definitions.

Convention: ``M[out, in]``.  For two-qubit gates the basis index is
``2*b(q0) + b(q1)``.  The paper names the fSim gate (Section 5.2) without
parameters; the circuits here use fSim(pi/2, pi/6):

    fSim(theta, phi) = [[1, 0,               0,               0         ],
                        [0, cos(theta),     -i sin(theta),    0         ],
                        [0, -i sin(theta),   cos(theta),      0         ],
                        [0, 0,               0,               e^{-i phi}]]

Single-qubit gates: H, and the square roots of X, Y and W = (X+Y)/sqrt(2)
with the convention (sqrt G)^2 = -i G.
"""
import math
import numpy as np
import rqcgen

_S = 1.0 / math.sqrt(2.0)

H_M = np.array([[1, 1], [1, -1]], dtype=np.complex128) * _S
SQRT_X_M = np.array([[1, -1j], [-1j, 1]], dtype=np.complex128) * _S
SQRT_Y_M = np.array([[1, -1], [1, 1]], dtype=np.complex128) * _S
_SQRT_I = np.exp(1j * math.pi / 4)       # sqrt(i)
_SQRT_MI = np.exp(-1j * math.pi / 4)     # sqrt(-i)
SQRT_W_M = np.array([[1, -_SQRT_I], [_SQRT_MI, 1]], dtype=np.complex128) * _S


def fsim(theta: float, phi: float) -> np.ndarray:
    c = math.cos(theta)
    s = math.sin(theta)
    return np.array([[1, 0, 0, 0],
                     [0, c, -1j * s, 0],
                     [0, -1j * s, c, 0],
                     [0, 0, 0, np.exp(-1j * phi)]], dtype=np.complex128)


def gate_matrix(g) -> np.ndarray:
    """Matrix of an ``rqcgen.Gate``: 2x2 or 4x4 complex128."""
    k = g.kind
    if k == rqcgen.H:
        return H_M
    if k == rqcgen.SQRT_X:
        return SQRT_X_M
    if k == rqcgen.SQRT_Y:
        return SQRT_Y_M
    if k == rqcgen.SQRT_W:
        return SQRT_W_M
    if k == rqcgen.FSIM:
        return fsim(g.theta, g.phi)
    if k in (rqcgen.U1, rqcgen.U2):
        m = np.asarray(g.u, dtype=np.complex128)
        want = (2, 2) if k == rqcgen.U1 else (4, 4)
        if m.shape != want:
            raise ValueError(f"explicit gate matrix must be {want}")
        return m
    raise ValueError(f"unknown gate kind {k}")
