"""Pins of the oracle's full-definition reconstruction (Eq. 1): brute-force
state-vector simulation of the uncut circuit, closed forms and invariants."""
import numpy as np
import pytest

from oracle import attribution as at
from oracle import cutmap
from oracle import reconstruct as rc
from oracle import statevector as sv
from workloads import circuits as wc
from workloads import synthetic as syn


def reconstruct_from_circuit(cc, form="definition"):
    subs = cc.subcircuits()
    E = [at.attribute(s, sv.variant_probabilities(s)) for s in subs]
    if form == "definition":
        p = rc.fd_definition(subs, E)
    else:
        p = rc.fd_contract(subs, E)
    return rc.apply_out_perm(p, cc.out_perm()), subs, E


def test_8_qubit_one_cut_matches_statevector():
    cc = wc.two_way_circuit_8q(seed=0)
    subs = cc.subcircuits()
    assert [s.width for s in subs] == [5, 4]
    p, _, _ = reconstruct_from_circuit(cc)
    ref = sv.probabilities(8, cc.ops)
    assert np.max(np.abs(p - ref)) < 1e-12
    assert p.sum() == pytest.approx(1.0, abs=1e-12)


def test_20_qubit_four_cuts_matches_statevector():
    cc = wc.two_way_circuit_20q(seed=1)
    subs = cc.subcircuits()
    assert [s.width for s in subs] == [12, 12]
    assert [len(cutmap.outputs(s)) for s in subs] == [10, 10]
    assert cc.out_perm() == [0, 1, 2, 3, 4, 5, 6, 7, 10, 11, 8, 9] + list(range(12, 20))
    p, _, _ = reconstruct_from_circuit(cc, form="contract")
    ref = sv.probabilities(20, cc.ops)
    assert np.max(np.abs(p - ref)) < 1e-12


def _random_cases(count, seed0=100):
    out, seed = [], seed0
    while len(out) < count:
        rng = np.random.default_rng(seed)
        seed += 1
        n = int(rng.integers(3, 8))
        n_sub = int(rng.integers(2, 4))
        n_cuts = int(rng.integers(1, 4))
        cc = wc.random_cut_circuit(rng, n, n_sub, n_cuts, depth=5)
        if cc is None or len(cc.cuts) == 0:
            continue
        if sum(len(cutmap.outputs(s)) for s in cc.subcircuits()) != n:
            continue
        out.append(cc)
    return out


@pytest.mark.parametrize("cc", _random_cases(24))
def test_random_cut_circuits_match_statevector(cc):
    p, subs, E = reconstruct_from_circuit(cc)
    ref = sv.probabilities(cc.n_qubits, cc.ops)
    assert np.max(np.abs(p - ref)) < 1e-12
    # the other two forms of Eq. 1 agree with the literal sum
    q = rc.fd_definition(subs, E)
    assert np.max(np.abs(rc.fd_contract(subs, E) - q)) < 1e-13
    bins = np.arange(q.size)[::3]
    assert np.max(np.abs(rc.fd_per_bin(subs, E, bins) - q[bins])) < 1e-13


def test_random_cases_cover_double_cuts_and_both_directions():
    cases = _random_cases(24)
    both_roles = any(any(i != -1 and m != -1 for i, m in zip(s.init_cut, s.meas_cut))
                     for cc in cases for s in cc.subcircuits())
    mixed = any(any(any(i != -1 for i in s.init_cut) and any(m != -1 for m in s.meas_cut)
                    for s in cc.subcircuits()) for cc in cases)
    three = any(cc.n_subcircuits == 3 for cc in cases)
    assert both_roles and mixed and three


def test_no_cuts_reduces_to_kron():
    rng = np.random.default_rng(7)
    ops = [wc.Op("u", (q,), wc.haar_u2(rng)) for q in range(4)]
    ops += [wc.Op("cz", (0, 1)), wc.Op("cz", (2, 3))]
    ops += [wc.Op("u", (q,), wc.haar_u2(rng)) for q in range(4)]
    cc = wc.CutCircuit(4, ops, [], {(0, 0): 0, (1, 0): 0, (2, 0): 1, (3, 0): 1})
    p, subs, E = reconstruct_from_circuit(cc)
    assert np.allclose(p, np.kron(E[0][0], E[1][0]), atol=1e-15)
    assert np.max(np.abs(p - sv.probabilities(4, cc.ops))) < 1e-13


def test_identity_rows_only_give_scaled_kron():
    rng = np.random.default_rng(8)
    cm = syn.chain_cutmap([2, 1], [3, 2, 3])
    ks = syn.chain_ks([2, 1], 3)
    E = [rng.standard_normal((4 ** k, 2 ** 3 if c != 1 else 4)) for c, k in enumerate(ks)]
    for e in E:
        e[1:] = 0.0
    p = rc.fd_definition(cm, E)
    assert np.allclose(p, 2.0 ** -3 * np.kron(np.kron(E[0][0], E[1][0]), E[2][0]), atol=1e-15)


def test_synthetic_sum_closed_form():
    # sum_b p = 2^-K sum_l prod_c rowsum_c(l_c): every output bit summed out
    cm, E = syn.chain_instance(3, [2, 2], [4, 3, 4])
    p = rc.fd_definition(cm, E)
    K = 4
    total = 0.0
    import itertools
    for labels in itertools.product(range(4), repeat=K):
        t = 1.0
        for s, e in zip(cm, E):
            t *= e[cutmap.local_label(s, labels)].sum()
        total += t
    assert p.sum() == pytest.approx(total * 2.0 ** -K, rel=1e-12)


def test_subcircuit_marginal():
    # summing p over subcircuit 0's outputs = reconstruction with subcircuit
    # 0's entries replaced by their row sums (a subcircuit without outputs)
    cm, E = syn.chain_instance(4, [2, 1], [3, 4, 2])
    p = rc.fd_definition(cm, E).reshape(2 ** 3, 2 ** 4 * 2 ** 2)
    cm0 = syn.chain_cutmap([2, 1], [0, 4, 2])
    q = rc.fd_definition(cm0, [E[0].sum(axis=1, keepdims=True), E[1], E[2]])
    assert np.max(np.abs(p.sum(axis=0) - q)) < 1e-15


def test_cut_relabeling_invariance():
    rng = np.random.default_rng(1)
    # three-subcircuit random case with several cuts
    for cc in _random_cases(6, seed0=500):
        subs = cc.subcircuits()
        V = [sv.variant_probabilities(s) for s in subs]
        p = rc.fd_definition(subs, [at.attribute(s, v) for s, v in zip(subs, V)])
        K = cutmap.total_cuts(subs)
        pi = rng.permutation(K)
        relab = [(s.width, [int(pi[c]) if c != -1 else -1 for c in s.init_cut],
                  [int(pi[c]) if c != -1 else -1 for c in s.meas_cut]) for s in subs]
        q = rc.fd_definition(relab, [at.attribute(s, v) for s, v in zip(relab, V)])
        assert np.max(np.abs(p - q)) < 1e-13


def test_integer_entries_exact_across_forms():
    rng = np.random.default_rng(11)
    cm = syn.chain_cutmap([1, 2], [3, 2, 3])
    ks = syn.chain_ks([1, 2], 3)
    E = [syn.integer_entries(rng, k, n) for k, n in zip(ks, [3, 2, 3])]
    a = rc.fd_definition(cm, E)
    b = rc.fd_contract(cm, E)
    c = rc.fd_per_bin(cm, E, np.arange(a.size))
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_dirichlet_generator_columns_and_torch_agree():
    full = syn.dirichlet_entries(9, 1, 2, 6)
    assert full[0].sum() == pytest.approx(1.0)
    assert np.all(np.abs(full[1:]) <= full[0][None, :] + 1e-300)
    cols = np.array([0, 5, 17, 63])
    assert np.array_equal(syn.entries_columns(9, 1, 2, 6, cols), full[:, cols])
    import torch
    t = syn.entries_torch(9, 1, 2, 6, "cpu", chunk_rows=3).numpy()
    assert np.array_equal(t, full)
