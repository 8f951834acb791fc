"""Pins of the oracle's state-vector simulator (Section 2) against an
independent dense-matrix construction and closed-form states."""
import numpy as np
import pytest

from oracle import statevector as sv
from workloads.circuits import H, Op, haar_u2

pytestmark = pytest.mark.filterwarnings("ignore")


def dense_unitary(n, ops):
    """The whole circuit as one 2^n x 2^n matrix: each gate is a Kronecker
    product of 2x2 factors in qubit order (qubit 0 leftmost = most
    significant), CZ is the diagonal matrix with -1 where both bits are 1."""
    U = np.eye(2 ** n, dtype=complex)
    for op in ops:
        if op.name == "u":
            f = [np.eye(2)] * n
            f = list(f)
            f[op.qubits[0]] = op.matrix
            G = np.array([[1.0]])
            for m in f:
                G = np.kron(G, m)
        else:
            a, b = op.qubits
            d = np.ones(2 ** n, dtype=complex)
            for x in range(2 ** n):
                if (x >> (n - 1 - a)) & 1 and (x >> (n - 1 - b)) & 1:
                    d[x] = -1
            G = np.diag(d)
        U = G @ U
    return U


@pytest.mark.parametrize("seed", range(6))
def test_simulate_matches_dense_unitary(seed):
    rng = np.random.default_rng(seed)
    n = 2 + seed % 4
    ops = []
    for _ in range(12):
        if rng.random() < 0.6 or n < 2:
            ops.append(Op("u", (int(rng.integers(n)),), haar_u2(rng)))
        else:
            a, b = rng.choice(n, 2, replace=False)
            ops.append(Op("cz", (int(a), int(b))))
    psi = sv.simulate(n, ops)
    ref = dense_unitary(n, ops)[:, 0]
    assert np.max(np.abs(psi - ref)) < 1e-12


def test_qubit_zero_is_most_significant():
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    p = sv.probabilities(3, [Op("u", (0,), X)])
    assert p[4] == pytest.approx(1.0)
    p = sv.probabilities(3, [Op("u", (2,), X)])
    assert p[1] == pytest.approx(1.0)


def test_bell_and_ghz_closed_forms():
    cnot01 = [Op("u", (1,), H), Op("cz", (0, 1)), Op("u", (1,), H)]
    p = sv.probabilities(2, [Op("u", (0,), H)] + cnot01)
    assert np.allclose(p, [0.5, 0, 0, 0.5], atol=1e-15)
    cnot12 = [Op("u", (2,), H), Op("cz", (1, 2)), Op("u", (2,), H)]
    ops = [Op("u", (0,), H)]
    ops += [Op("u", (1,), H), Op("cz", (0, 1)), Op("u", (1,), H)] + cnot12
    p = sv.probabilities(3, ops)
    ref = np.zeros(8)
    ref[0] = ref[7] = 0.5
    assert np.allclose(p, ref, atol=1e-15)


def test_haar_u2_is_unitary():
    rng = np.random.default_rng(5)
    for _ in range(20):
        u = haar_u2(rng)
        assert np.allclose(u.conj().T @ u, np.eye(2), atol=1e-14)


def test_variant_basis_changes_measure_pauli_eigenstates():
    # the +1 eigenstate of each basis maps to outcome 0
    plus_y = sv.KETPI
    for basis, ket in ((0, sv.KET0), (1, sv.KETP), (2, plus_y)):
        out = sv.BASIS_CHANGE[basis] @ ket
        assert abs(out[0]) ** 2 == pytest.approx(1.0)
