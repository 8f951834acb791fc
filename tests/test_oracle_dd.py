"""Pins of the oracle's dynamic definition (Algorithm 1): bins against
brute-force sums of the full distribution, the all-active / all-merged
limits, parent/child consistency, and the hidden-string search of Section
4.3 (sparse output found in O(n) recursions)."""
import numpy as np
import pytest

from oracle import attribution as at
from oracle import cutmap
from oracle import dd
from oracle import reconstruct as rc
from oracle import statevector as sv
from workloads import circuits as wc
from workloads import synthetic as syn


def brute_force_bins(subs, p_concat, states):
    """Bins as sums of full-distribution entries: loop over every state, keep
    those matching the zoomed values, accumulate by the active bits."""
    ns = [len(cutmap.outputs(s)) for s in subs]
    n = sum(ns)
    n_act = sum(len(st.active) for st in states)
    out = np.zeros(2 ** n_act)
    for x in range(2 ** n):
        bits = [(x >> (n - 1 - i)) & 1 for i in range(n)]
        ok, idx, off = True, 0, 0
        for st, nc in zip(states, ns):
            mine = bits[off:off + nc]
            off += nc
            for pos, v in st.fixed.items():
                if mine[pos] != v:
                    ok = False
            for pos in sorted(st.active):
                idx = 2 * idx + mine[pos]
        if ok:
            out[idx] += p_concat[x]
    return out


def random_states(rng, ns):
    states = []
    for n in ns:
        roles = rng.integers(0, 3, size=n)   # 0 active, 1 merged, 2 fixed
        st = dd.SubState([int(i) for i in np.flatnonzero(roles == 0)],
                         [int(i) for i in np.flatnonzero(roles == 1)],
                         {int(i): int(rng.integers(2)) for i in np.flatnonzero(roles == 2)})
        states.append(st)
    return states


@pytest.mark.parametrize("seed", range(8))
def test_bins_equal_brute_force_sums(seed):
    rng = np.random.default_rng(seed)
    bonds = [int(rng.integers(0, 3)), int(rng.integers(1, 3))]
    ns = [3, 2 + int(rng.integers(0, 2)), 3]
    cm = syn.chain_cutmap(bonds, ns)
    E = [syn.integer_entries(rng, k, n) for k, n in zip(syn.chain_ks(bonds, 3), ns)]
    p = rc.fd_definition(cm, E)
    states = random_states(rng, ns)
    assert np.array_equal(dd.bins_of(cm, E, states), brute_force_bins(cm, p, states))


def test_all_active_is_fd_and_all_merged_is_total():
    cm, E = syn.chain_instance(5, [2, 1], [3, 3, 2])
    p = rc.fd_definition(cm, E)
    act = [dd.SubState(list(range(n)), [], {}) for n in (3, 3, 2)]
    assert np.max(np.abs(dd.bins_of(cm, E, act) - p)) < 1e-15
    mer = [dd.SubState([], list(range(n)), {}) for n in (3, 3, 2)]
    tot = dd.bins_of(cm, E, mer)
    assert tot.shape == (1,) and tot[0] == pytest.approx(p.sum(), abs=1e-15)


def test_physical_circuit_dd_matches_statevector_and_children_sum_to_parent():
    cc = wc.two_way_circuit_8q(seed=0)
    subs = cc.subcircuits()
    E = [at.attribute(s, sv.variant_probabilities(s)) for s in subs]
    p = rc.fd_definition(subs, E)
    ns = [len(cutmap.outputs(s)) for s in subs]
    st0 = dd.initial_states(subs, [2, 1])
    recs = dd.run(subs, E, st0, [2, 1], R=4)
    assert len(recs) == 4
    for r, rec in enumerate(recs):
        ref = brute_force_bins(subs, p, rec["states"])
        assert np.max(np.abs(rec["bins"] - ref)) < 1e-14
        # L is sorted and popped from its head
        vals = [v for (v, _, _) in rec["L"]]
        assert vals == sorted(vals, reverse=True)
        if r > 0:
            parent = recs[r - 1]["popped"]
            assert rec["bins"].sum() == pytest.approx(parent[0], abs=1e-14)
    assert ns == [4, 4]


def test_integer_entries_zoom_path_and_ties():
    rng = np.random.default_rng(21)
    cm = syn.chain_cutmap([1, 1], [3, 3, 3])
    E = [syn.integer_entries(rng, k, 3, lo=0, hi=2) for k in syn.chain_ks([1, 1], 3)]
    p = rc.fd_definition(cm, E)
    recs = dd.run(cm, E, dd.initial_states(cm, [1, 1, 1]), [1, 1, 1], R=3)
    for rec in recs:
        assert np.array_equal(rec["bins"], brute_force_bins(cm, p, rec["states"]))
        # popped = best of L under (value desc, recursion asc, index asc)
        if rec["popped"] is not None:
            L_before = [rec["popped"]] + rec["L"]
            key = lambda e: (-e[0], e[1], e[2])
            assert min(L_before, key=key) == rec["popped"]


def test_hidden_string_found_in_linear_recursions():
    secret = [1, 0, 1, 1, 0, 0, 1, 0, 1]
    groups = [[0, 1, 2], [3, 4, 5], [6, 7, 8]]
    cc = wc.hidden_string_circuit(secret, groups)
    subs = cc.subcircuits()
    E = [at.attribute(s, sv.variant_probabilities(s)) for s in subs]
    ns = [len(cutmap.outputs(s)) for s in subs]
    assert ns == [3, 3, 4]
    M = [1, 1, 1]
    recs = dd.run(subs, E, dd.initial_states(subs, M), M, R=4)
    # each recursion resolves one qubit per subcircuit: 4 recursions resolve all 10
    last = recs[-1]
    assert not any(st.merged for st in last["states"])
    best = int(np.argmax(last["bins"]))
    assert last["bins"][best] == pytest.approx(1.0, abs=1e-12)
    # reassemble the full state of the winning bin
    bits = []
    off = sum(len(st.active) for st in last["states"])
    for st, n in zip(last["states"], ns):
        a = len(st.active)
        off -= a
        val = (best >> off) & ((1 << a) - 1)
        full = dict(st.fixed)
        for i, pos in enumerate(sorted(st.active)):
            full[pos] = (val >> (a - 1 - i)) & 1
        bits += [full[i] for i in range(n)]
    perm = cc.out_perm()
    state = [0] * len(perm)
    for i, q in enumerate(perm):
        state[q] = bits[i]
    assert state == secret + [1]


# --- breadth-first query (dense outputs) --------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_bfs_nodes_are_brute_force_bins_and_refine_their_parent(seed):
    """Every node's bins are brute-force sums of the full distribution over
    its labels; a child's bins partition the parent bin it zooms into; each
    level zooms into the best candidates of the level above (value desc,
    then parent, then bin) and every node's candidates are its best bins."""
    rng = np.random.default_rng(40 + seed)
    bonds = [int(rng.integers(1, 3)), int(rng.integers(1, 3))]
    ns = [4, 3, 4]
    cm = syn.chain_cutmap(bonds, ns)
    E = [syn.integer_entries(rng, k, n, lo=0, hi=3) for k, n in zip(syn.chain_ks(bonds, 3), ns)]
    p = rc.fd_definition(cm, E)
    M = [1, 1, 2]
    W = 3
    nodes = dd.run_bfs(cm, E, dd.initial_states(cm, M), M, levels=3, width=W)
    assert nodes[0]["level"] == 0 and nodes[0]["parent"] == -1
    by_level = {}
    for k, nd in enumerate(nodes):
        by_level.setdefault(nd["level"], []).append(k)
        assert np.array_equal(nd["bins"], brute_force_bins(cm, p, nd["states"]))
        if nd["parent"] >= 0:
            par = nodes[nd["parent"]]
            assert par["level"] == nd["level"] - 1
            assert nd["total"] == par["bins"][nd["parent_bin"]]   # integer sums: exact
        # candidates: the W best bins (value desc, index asc) of a node that still merges
        if any(st.merged for st in nd["states"]):
            want = sorted(range(len(nd["bins"])), key=lambda i: (-nd["bins"][i], i))[:W]
            assert [i for (_, i) in nd["candidates"]] == want
    for lv in range(1, max(by_level) + 1):
        pool = [(v, k, i) for k in by_level[lv - 1] for (v, i) in nodes[k]["candidates"]]
        pool.sort(key=lambda e: (-e[0], e[1], e[2]))
        got = [(nodes[k]["parent"], nodes[k]["parent_bin"]) for k in by_level[lv]]
        assert got == [(k, i) for (_, k, i) in pool[:W]]
    assert len(by_level) == 3 and len(by_level[1]) == W


def test_bfs_reaches_full_definition_of_the_heaviest_region():
    """With nothing left merged after enough levels, the deepest nodes'
    bins are single probabilities of the full distribution."""
    cm, E = syn.chain_instance(9, [1, 1], [3, 3, 3])
    p = rc.fd_definition(cm, E)
    M = [1, 1, 1]
    nodes = dd.run_bfs(cm, E, dd.initial_states(cm, M), M, levels=3, width=2)
    deep = [nd for nd in nodes if nd["level"] == 2]
    assert deep
    for nd in deep:
        assert not any(st.merged for st in nd["states"])
        assert not nd["candidates"]
        ref = brute_force_bins(cm, p, nd["states"])
        assert np.max(np.abs(nd["bins"] - ref)) < 1e-15
    # a level with no candidates ends the query
    more = dd.run_bfs(cm, E, dd.initial_states(cm, M), M, levels=6, width=2)
    assert max(nd["level"] for nd in more) == 2
