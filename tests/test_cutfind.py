"""The exact cut search (Section 4.1's clustering of two-qubit gates and
its multiplication-count objective) against hand-worked cases, against the
cut structure of circuits built by the workload generator, and through the
C ABI against the oracle's exhaustive search.  Host only."""
import numpy as np
import pytest

from oracle import attribution as at
from oracle import cutfind as cf
from oracle import reconstruct as rc
from oracle import statevector as sv
from workloads import circuits as wc


def cq():
    import paper_2205_05836_amd as m
    return m


def test_hand_worked_chain_of_four():
    """CZ(0,1) CZ(1,2) CZ(2,3) on devices of 3 qubits.  {g0,g1}|{g2} cuts q2
    once: widths 3 and 2, outputs 2 and 2, L = 4 * 2^2 * 2^2 = 64.
    {g0}|{g1,g2} cuts q1: outputs 1 and 3, also 64; {g0,g2}|{g1} needs two
    cuts.  The tie goes to the label string 001."""
    gates = [(0, 1), (1, 2), (2, 3)]
    assert cf.structure(4, gates, (0, 0, 1)) == (1, [3, 2], [2, 2])
    assert cf.structure(4, gates, (0, 1, 1)) == (1, [2, 3], [1, 3])
    assert cf.structure(4, gates, (0, 1, 0)) == (2, [4, 2], [3, 1])
    want = dict(cluster=[0, 0, 1], cost=64.0, n_cuts=1, n_subcircuits=2)
    assert cf.best_clustering(4, gates, 3, 5) == want
    assert cq().cq_find_cuts(4, gates, 3) == want
    # a device that holds the whole circuit needs no cut
    assert cq().cq_find_cuts(4, gates, 4) == dict(cluster=[0, 0, 0], cost=0.0, n_cuts=0,
                                                   n_subcircuits=1)


def test_cost_of_three_subcircuits():
    """Outputs (1, 3, 2), K cuts: sorted (1, 2, 3) gives 4^K (2^3 + 2^6)."""
    assert cf.cost(2, [1, 3, 2]) == 16 * (8 + 64)
    assert cf.cost(0, [5]) == 0.0


@pytest.mark.parametrize("which", ["8q", "20q"])
def test_structure_matches_generated_cut_circuits(which):
    """The clustering that the generator's cut circuits realise: K, widths
    and outputs from the oracle's structure() against the subcircuits the
    generator builds independently."""
    cc = wc.two_way_circuit_8q(0) if which == "8q" else wc.two_way_circuit_20q(1)
    pairs, labels = [], []
    for i, op in enumerate(cc.ops):
        if op.name == "cz":
            q = op.qubits[0]
            pairs.append(tuple(op.qubits))
            labels.append(cc.assignment[(q, cc.segment(q, i))])
    # every cut of these circuits sits between two two-qubit gates on its wire
    cuts, width, outputs = cf.structure(cc.n_qubits, pairs, cf.canonical(labels))
    subs = cc.subcircuits()
    order = cf.canonical(labels)
    first = {}
    for raw, can in zip(labels, order):
        first.setdefault(raw, can)
    assert cuts == len(cc.cuts)
    for raw, spec in enumerate(subs):
        c = first[raw]
        assert width[c] == spec.width
        assert outputs[c] == sum(1 for m in spec.meas_cut if m == -1)


def _random_problem(rng):
    n = int(rng.integers(3, 7))
    g = int(rng.integers(n - 1, 8))
    # a spanning chain keeps every qubit busy, then random pairs
    perm = rng.permutation(n)
    pairs = [(int(perm[i]), int(perm[i + 1])) for i in range(n - 1)]
    while len(pairs) < g:
        a, b = rng.choice(n, size=2, replace=False)
        pairs.append((int(a), int(b)))
    order = rng.permutation(len(pairs))
    return n, [pairs[i] for i in order]


@pytest.mark.parametrize("seed", range(24))
def test_library_matches_exhaustive_oracle(seed):
    rng = np.random.default_rng(seed)
    n, gates = _random_problem(rng)
    max_width = int(rng.integers(2, n + 1))
    max_sub = int(rng.integers(2, 5))
    want = cf.best_clustering(n, gates, max_width, max_sub)
    if want is None:
        with pytest.raises(cq().CQError):
            cq().cq_find_cuts(n, gates, max_width, max_sub)
        return
    got = cq().cq_find_cuts(n, gates, max_width, max_sub)
    assert got == want


def test_rejects_bad_problems():
    m = cq()
    with pytest.raises(m.CQError):
        m.cq_find_cuts(3, [(0, 1)], 3)              # qubit 2 idle
    with pytest.raises(m.CQError):
        m.cq_find_cuts(2, [(0, 0)], 3)              # equal qubits
    with pytest.raises(m.CQError):
        m.cq_find_cuts(2, [(0, 1)] * 17, 3)         # too many gates
    with pytest.raises(m.CQError):
        m.cq_find_cuts(3, [(0, 1), (1, 2)], 1)      # nothing fits one qubit


def test_sixteen_gate_brickwork_finishes():
    """The largest search (16 gates, five clusters) on a 9-qubit brickwork
    for 5-qubit devices: a feasible clustering whose reported cost agrees
    with the oracle's formula."""
    pairs = [(i, i + 1) for t in range(4) for i in range(t % 2, 8, 2)]
    assert len(pairs) == 16
    got = cq().cq_find_cuts(9, pairs, 5)
    cuts, width, outputs = cf.structure(9, pairs, tuple(got["cluster"]))
    assert max(width) <= 5 and cuts == got["n_cuts"]
    assert got["cost"] == cf.cost(cuts, outputs)


@pytest.mark.parametrize("seed", range(4))
def test_found_cuts_reconstruct_the_circuit(seed):
    """The library's cut search on a random 6-qubit circuit for 4-qubit
    devices; the circuit cut where it says, simulated per variant and
    reconstructed by the oracle (Eq. 1), equals the uncut state vector, and
    the cut circuit's subcircuits fit the device."""
    rng = np.random.default_rng(100 + seed)
    n = 6
    ops = []
    chain = rng.permutation(n)
    pairs = [(int(chain[i]), int(chain[i + 1])) for i in range(n - 1)]
    pairs += [tuple(int(x) for x in rng.choice(n, size=2, replace=False)) for _ in range(3)]
    for a, b in pairs:
        ops.append(wc.Op("u", (a,), wc.haar_u2(rng)))
        ops.append(wc.Op("u", (b,), wc.haar_u2(rng)))
        ops.append(wc.Op("cz", (a, b)))
    ops += [wc.Op("u", (q,), wc.haar_u2(rng)) for q in range(n)]
    found = cq().cq_find_cuts(n, ops, max_width=4, max_subcircuits=3)
    cc = wc.cut_circuit_from_clusters(n, ops, found["cluster"])
    subs = cc.subcircuits()
    assert found["n_cuts"] >= 1                   # six qubits cannot fit one device of four
    assert len(cc.cuts) == found["n_cuts"] and len(subs) == found["n_subcircuits"]
    assert max(s.width for s in subs) <= 4
    E = [at.attribute(s, sv.variant_probabilities(s)) for s in subs]
    p = rc.apply_out_perm(rc.fd_definition(subs, E), cc.out_perm())
    assert np.max(np.abs(p - sv.probabilities(n, ops))) < 1e-12
