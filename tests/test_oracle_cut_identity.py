"""Pins of the oracle's cut decomposition (Section 3.1): the single-qubit
Pauli identity, the hand-derived worked example and the structural counts of
the paper's Fig. 2 example."""
import json
import os

import numpy as np
import pytest

from oracle import attribution as at
from oracle import reconstruct as rc
from oracle import statevector as sv
from workloads.circuits import H, CutCircuit, Op, haar_u2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

PAULI = (np.eye(2, dtype=complex),
         np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex),
         np.array([[1, 0], [0, -1]], dtype=complex))


def random_rho(rng):
    a = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    r = a @ a.conj().T
    return r / np.trace(r)


def test_init_coefficients_rebuild_pauli_operators():
    for label in range(4):
        op = sum(at.ALPHA[label][j] * np.outer(sv.INIT_STATES[j], sv.INIT_STATES[j].conj())
                 for j in range(4))
        assert np.allclose(op, PAULI[label], atol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_measured_expectations_and_single_cut_identity(seed):
    rho = random_rho(np.random.default_rng(seed))
    rebuilt = np.zeros((2, 2), dtype=complex)
    for label in range(4):
        B = sv.BASIS_CHANGE[at.BASIS_OF[label]]
        probs = np.real(np.diag(B @ rho @ B.conj().T))
        expval = sum(at.sign(label, m) * probs[m] for m in range(2))
        assert expval == pytest.approx(np.real(np.trace(rho @ PAULI[label])), abs=1e-14)
        op = sum(at.ALPHA[label][j] * np.outer(sv.INIT_STATES[j], sv.INIT_STATES[j].conj())
                 for j in range(4))
        rebuilt += 0.5 * expval * op
    assert np.max(np.abs(rebuilt - rho)) < 1e-14


def bell_cut_circuit():
    ops = [Op("u", (0,), H), Op("u", (1,), H), Op("cz", (0, 1)), Op("u", (1,), H)]
    return CutCircuit(2, ops, [(0, 0)], {(0, 0): 0, (0, 1): 1, (1, 0): 1})


def test_golden_bell_cut_worked_example():
    with open(os.path.join(GOLDEN, "bell_cut.json")) as f:
        g = json.load(f)
    cc = bell_cut_circuit()
    subs = cc.subcircuits()
    V0 = sv.variant_probabilities(subs[0])
    V1 = sv.variant_probabilities(subs[1])
    assert np.allclose(V0, g["variants_sub0"], atol=1e-15)
    assert np.allclose(V1, g["variants_sub1"], atol=1e-15)
    E0, E1 = at.attribute(subs[0], V0), at.attribute(subs[1], V1)
    assert np.allclose(E0, g["entries_sub0"], atol=1e-15)
    assert np.allclose(E1, g["entries_sub1"], atol=1e-15)
    p = rc.apply_out_perm(rc.fd_definition(subs, [E0, E1]), cc.out_perm())
    assert np.allclose(p, g["p"], atol=1e-15)
    assert np.allclose(p, sv.probabilities(2, cc.ops), atol=1e-15)


def test_fig2_structure_counts():
    with open(os.path.join(GOLDEN, "fig2_structure.json")) as f:
        g = json.load(f)
    rng = np.random.default_rng(2)
    ops = [Op("u", (q,), haar_u2(rng)) for q in range(5)]
    ops += [Op("cz", (0, 1)), Op("cz", (1, 2))]
    cut_pos = len(ops) - 1
    ops += [Op("cz", (2, 3)), Op("cz", (3, 4))]
    ops += [Op("u", (q,), haar_u2(rng)) for q in range(5)]
    assign = {(0, 0): 0, (1, 0): 0, (2, 0): 0, (2, 1): 1, (3, 0): 1, (4, 0): 1}
    cc = CutCircuit(5, ops, [(2, cut_pos)], assign)
    subs = cc.subcircuits()
    assert cc.n_qubits == g["n_qubits"] and len(cc.cuts) == g["n_cuts"]
    assert [s.width for s in subs] == g["subcircuit_widths"]
    V0, V1 = sv.variant_probabilities(subs[0]), sv.variant_probabilities(subs[1])
    assert V0.shape[0] * V0.shape[1] == g["upstream_variants"]
    assert V1.shape[0] * V1.shape[1] == g["downstream_variants"]
    assert 4 ** len(cc.cuts) == g["kronecker_products"]
    E = [at.attribute(s, V) for s, V in zip(subs, (V0, V1))]
    p = rc.apply_out_perm(rc.fd_definition(subs, E), cc.out_perm())
    assert np.max(np.abs(p - sv.probabilities(5, cc.ops))) < 1e-13
