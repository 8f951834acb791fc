"""Entry attribution: subcircuit variant probabilities -> entries p_{i,k}.
Test infrastructure only.

Section 3.1 decomposes the qubit state crossing each cut into the Pauli bases
{I, X, Y, Z}; the physics is in the work the paper cites for it.  Writing a
single-qubit state as rho = 1/2 sum_sigma Tr(rho sigma) sigma, a cut labelled
sigma contributes

* at its upstream end, the expectation of sigma: measure in sigma's
  eigenbasis (I and Z: computational basis; X: after H; Y: after S^dagger H)
  and weight outcome m by the eigenvalue, +1 for I and (-1)^m otherwise;
* at its downstream end, the operator sigma itself, expanded over the four
  preparable states: I = |0><0| + |1><1|, Z = |0><0| - |1><1|,
  X = 2|+><+| - I, Y = 2|+i><+i| - I.

So with label digits I=0, X=1, Y=2, Z=3, init digits |0>,|1>,|+>,|+i> = 0..3
and basis digits Z, X, Y = 0..2:

  E[l][b] = sum_j prod_t ALPHA[l_t][j_t]
            * sum_m prod_u SIGN(l_u, m_u) * V[j][basis(l)][compose(b, m)]

where t runs over init slots, u over measured slots, b over the output bits
and m over the measured bits.  The 1/2 per cut is applied once, at the end of
reconstruction (2^-K).
"""
from __future__ import annotations

import itertools

import numpy as np

from . import cutmap

I, X, Y, Z = 0, 1, 2, 3

# ALPHA[label][init digit]: coefficient of each prepared state.
ALPHA = (
    (1.0, 1.0, 0.0, 0.0),    # I = |0><0| + |1><1|
    (-1.0, -1.0, 2.0, 0.0),  # X = 2|+><+| - I
    (-1.0, -1.0, 0.0, 2.0),  # Y = 2|+i><+i| - I
    (1.0, -1.0, 0.0, 0.0),   # Z = |0><0| - |1><1|
)
# Measurement basis digit used for a label (Z basis serves I and Z).
BASIS_OF = (0, 1, 2, 0)


def sign(label, m):
    return 1.0 if label == I else (-1.0 if m else 1.0)


def attribute(sub, V):
    """Entries of one subcircuit, shape (4^k, 2^n), from its variant
    probabilities V of shape (4^r, 3^o, 2^w) (layout as produced by
    ``statevector.variant_probabilities``)."""
    w, init, meas = cutmap.unpack(sub)
    ins, ms, outs = cutmap.init_slots(sub), cutmap.meas_slots(sub), cutmap.outputs(sub)
    cuts = cutmap.incident_cuts(sub)
    r, o, n, k = len(ins), len(ms), len(outs), len(cuts)
    V = np.asarray(V, dtype=np.float64)
    assert V.shape == (4 ** r, 3 ** o, 2 ** w)

    # compose(b, m): register outcome index for output bits b and measured
    # bits m, one index array over b per m.
    b = np.arange(2 ** n)
    compose = {}
    for m in itertools.product(range(2), repeat=o):
        x = np.zeros(2 ** n, dtype=np.int64)
        for i, s in enumerate(outs):
            x |= ((b >> (n - 1 - i)) & 1) << (w - 1 - s)
        for u, s in enumerate(ms):
            x |= m[u] << (w - 1 - s)
        compose[m] = x

    E = np.zeros((4 ** k, 2 ** n))
    for l in range(4 ** k):
        digit = {c: (l // 4 ** (k - 1 - p)) % 4 for p, c in enumerate(cuts)}
        l_init = [digit[init[s]] for s in ins]
        l_meas = [digit[meas[s]] for s in ms]
        beta = 0
        for lu in l_meas:
            beta = 3 * beta + BASIS_OF[lu]
        for ji, j in enumerate(itertools.product(range(4), repeat=r)):
            coef = 1.0
            for lt, jt in zip(l_init, j):
                coef *= ALPHA[lt][jt]
            if coef == 0.0:
                continue
            for m in itertools.product(range(2), repeat=o):
                sg = 1.0
                for lu, mu in zip(l_meas, m):
                    sg *= sign(lu, mu)
                E[l] += coef * sg * V[ji, beta, compose[m]]
    return E
