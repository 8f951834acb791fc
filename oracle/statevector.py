"""State-vector simulation (Section 2, the noiseless ground truth) and the
subcircuit variants of Section 3.1.  Test infrastructure only.

Qubit 0 is the most significant bit of a basis-state index.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import cutmap

KET0 = np.array([1, 0], dtype=complex)
KET1 = np.array([0, 1], dtype=complex)
KETP = np.array([1, 1], dtype=complex) / np.sqrt(2.0)
KETPI = np.array([1, 1j], dtype=complex) / np.sqrt(2.0)

# Initial states of a cut's downstream end, by init digit: |0>, |1>, |+>, |+i>.
INIT_STATES = (KET0, KET1, KETP, KETPI)

_H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2.0)
_SDG = np.array([[1, 0], [0, -1j]], dtype=complex)
# Rotations applied before a computational-basis measurement of a cut's
# upstream end, by basis digit: Z basis (nothing), X basis (H), Y basis (S^dagger then H).
BASIS_CHANGE = (np.eye(2, dtype=complex), _H, _H @ _SDG)


def product_state(kets):
    psi = np.array([1.0 + 0j])
    for k in kets:
        psi = np.kron(psi, k)
    return psi


def apply_1q(psi, n, q, u):
    t = psi.reshape((2,) * n)
    t = np.tensordot(u, t, axes=([1], [q]))
    t = np.moveaxis(t, 0, q)
    return t.reshape(-1)


def apply_cz(psi, n, a, b):
    t = psi.reshape((2,) * n).copy()
    idx = [slice(None)] * n
    idx[a] = 1
    idx[b] = 1
    t[tuple(idx)] *= -1
    return t.reshape(-1)


def simulate(n, ops, psi0=None):
    """Apply ``ops`` (Op with name 'u' or 'cz') to ``psi0`` (default |0..0>)."""
    psi = product_state([KET0] * n) if psi0 is None else np.asarray(psi0, dtype=complex)
    for op in ops:
        if op.name == "u":
            psi = apply_1q(psi, n, op.qubits[0], op.matrix)
        elif op.name == "cz":
            psi = apply_cz(psi, n, op.qubits[0], op.qubits[1])
        else:
            raise ValueError(op.name)
    return psi


def probabilities(n, ops, psi0=None):
    psi = simulate(n, ops, psi0)
    return np.abs(psi) ** 2


def variant_probabilities(spec):
    """All variants of one subcircuit (Section 3.1, Fig. 2: 4 initialisations
    per downstream cut end, 3 measurement bases per upstream cut end).

    Returns V with shape (4^r, 3^o, 2^w): V[j][beta][x] is the probability of
    register outcome x when init slot t (slot order) is prepared in
    INIT_STATES[j_t] and measured slot u is rotated by BASIS_CHANGE[beta_u]
    before the final computational-basis measurement.  Digit strings are
    read most significant first."""
    w = spec.width
    ins, ms = cutmap.init_slots(spec), cutmap.meas_slots(spec)
    r, o = len(ins), len(ms)
    V = np.zeros((4 ** r, 3 ** o, 2 ** w))
    for ji, j in enumerate(itertools.product(range(4), repeat=r)):
        kets = [KET0] * w
        for t, s in enumerate(ins):
            kets[s] = INIT_STATES[j[t]]
        psi = simulate(w, spec.ops, product_state(kets))
        for bi, beta in enumerate(itertools.product(range(3), repeat=o)):
            phi = psi
            for u, s in enumerate(ms):
                phi = apply_1q(phi, w, s, BASIS_CHANGE[beta[u]])
            V[ji, bi] = np.abs(phi) ** 2
    return V
