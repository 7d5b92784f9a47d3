"""Textbook spin matrices and exact exponentials for the oracle's pins.

Written from the definitions (paper, Sec. "Quantum mechanics background"):
spin-1/2 J = sigma / 2; spin-1 J_x, J_y, J_z in the basis |+1>, |0>, |-1>
and Q = diag(1, -2, 1) / 3.  Exact exponentials use an eigendecomposition of
the Hermitian generator, independent of the oracle's closed forms.
"""
import numpy as np

SX2 = np.array([[0, 1], [1, 0]], dtype=complex) / 2
SY2 = np.array([[0, -1j], [1j, 0]], dtype=complex) / 2
SZ2 = np.array([[1, 0], [0, -1]], dtype=complex) / 2

_r = 1 / np.sqrt(2)
SX3 = _r * np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], dtype=complex)
SY3 = _r * np.array([[0, -1j, 0], [1j, 0, -1j], [0, 1j, 0]], dtype=complex)
SZ3 = np.diag([1, 0, -1]).astype(complex)
Q3 = np.diag([1, -2, 1]).astype(complex) / 3


def generator(theta, dim):
    th = list(theta) + [0.0] * (4 - len(theta))
    if dim == 2:
        return th[0] * SX2 + th[1] * SY2 + th[2] * SZ2
    return th[0] * SX3 + th[1] * SY3 + th[2] * SZ3 + th[3] * Q3


def expmh(H):
    """exp(-i H) for Hermitian H via eigh."""
    w, V = np.linalg.eigh(H)
    return (V * np.exp(-1j * w)) @ V.conj().T


def exact_exp(theta, dim):
    return expmh(generator(theta, dim))


def d1(U2):
    """Spin-1 representation D^1 of an SU(2) matrix [[a, b], [c, d]] in the
    basis |+1>, |0>, |-1>."""
    a, b = U2[..., 0, 0], U2[..., 0, 1]
    c, d = U2[..., 1, 0], U2[..., 1, 1]
    s = np.sqrt(2)
    out = np.empty(U2.shape[:-2] + (3, 3), dtype=complex)
    out[..., 0, 0] = a * a
    out[..., 0, 1] = s * a * b
    out[..., 0, 2] = b * b
    out[..., 1, 0] = s * a * c
    out[..., 1, 1] = a * d + b * c
    out[..., 1, 2] = s * b * d
    out[..., 2, 0] = c * c
    out[..., 2, 1] = s * c * d
    out[..., 2, 2] = d * d
    return out


def d1_state(v):
    """Spin-1 coherent state of a spin-1/2 state (a, b): (a^2, sqrt2 ab, b^2)."""
    a, b = v[..., 0], v[..., 1]
    return np.stack([a * a, np.sqrt(2) * a * b, b * b], axis=-1)
