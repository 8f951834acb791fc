"""Dynamic definition (Section 4.3, Algorithm 1).  Test infrastructure only.

Each recursion labels every output qubit active, merged or zoomed (fixed).
Bins are indexed by the active qubits; a bin holds the sum of the
probabilities of all states that agree with it on the active qubits, have
the zoomed qubits at their fixed values and take any value on the merged
qubits.  The 2^{#active} bins are reconstructed, the R largest bins that
still contain merged qubits are appended to a list L, L is sorted and cut to
its R largest, and the head of L is popped and zoomed into next.

Readings where the algorithm is silent or ambiguous:

* Merging happens on the entries instead of on grouped shots: summing entry
  columns over the merged bits at the fixed values gives the same bins,
  because every entry is linear in the subcircuit's output distribution.
* Choice of active qubits: per subcircuit, the first ``max_active[c]`` qubits
  (output order, most significant first) that are merged in the bin being
  zoomed; recursion 0 takes explicit masks.
* L holds (value, recursion, bin index) and sorts by value descending, then
  recursion ascending, then bin index ascending; its capacity is R.  Values
  are signed and are never clipped.
* The loop ends after R recursions, or earlier when L is empty at the pop.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import cutmap
from .reconstruct import fd_contract


@dataclass
class SubState:
    """Labels of one subcircuit's outputs: ``active`` and ``merged`` are
    lists of output positions (0 = most significant), ``fixed`` maps an
    output position to its zoomed value."""

    active: list
    merged: list
    fixed: dict = field(default_factory=dict)

    def copy(self):
        return SubState(list(self.active), list(self.merged), dict(self.fixed))


def merge_entries(E, n, st: SubState):
    """E'[l][a] = sum over merged bits of E[l][state with active bits a,
    zoomed bits at their values, merged bits free]."""
    E = np.asarray(E)
    t = E.reshape((E.shape[0],) + (2,) * n)
    idx = [slice(None)] * (n + 1)
    for pos, v in st.fixed.items():
        idx[1 + pos] = v
    t = t[tuple(idx)]
    # remaining axes: row, then the non-fixed positions in order
    rest = [p for p in range(n) if p not in st.fixed]
    sum_axes = tuple(1 + rest.index(p) for p in st.merged)
    t = t.sum(axis=sum_axes) if sum_axes else t
    kept = [p for p in rest if p not in st.merged]
    assert kept == sorted(st.active)
    return t.reshape(E.shape[0], -1)


def bins_of(subs, entries, states):
    ns = [len(cutmap.outputs(s)) for s in subs]
    reduced = [merge_entries(E, n, st) for E, n, st in zip(entries, ns, states)]
    return fd_contract(subs, reduced)


def child_states(states, bin_index):
    """States describing one bin: its active bits become fixed."""
    out, shift = [], sum(len(st.active) for st in states)
    for st in states:
        a = len(st.active)
        shift -= a
        bits = (bin_index >> shift) & ((1 << a) - 1)
        ch = st.copy()
        for i, p in enumerate(sorted(st.active)):
            ch.fixed[p] = (bits >> (a - 1 - i)) & 1
        ch.active = []
        out.append(ch)
    return out


def zoom(states, max_active):
    """Next recursion's labels for a popped bin."""
    out = []
    for st, m in zip(states, max_active):
        merged = sorted(st.merged)
        out.append(SubState(merged[:m], merged[m:], dict(st.fixed)))
    return out


def initial_states(subs, max_active):
    out = []
    for s, m in zip(subs, max_active):
        n = len(cutmap.outputs(s))
        out.append(SubState(list(range(min(m, n))), list(range(min(m, n), n)), {}))
    return out


def run(subs, entries, states0, max_active, R):
    """Algorithm 1.  Returns a list of per-recursion records:
    dict(states, bins, L (after update), popped (value, rec, index) or None)."""
    L = []
    records = []
    states = states0
    r = 0
    while r < R:
        bins = bins_of(subs, entries, states)
        has_merged = any(st.merged for st in states)
        if has_merged:
            order = sorted(range(len(bins)), key=lambda i: (-bins[i], i))[:R]
            for i in order:
                L.append((float(bins[i]), r, i, child_states(states, i)))
        L.sort(key=lambda e: (-e[0], e[1], e[2]))
        L = L[:R]
        rec = dict(states=[st.copy() for st in states], bins=bins,
                   L=[(v, rr, i) for (v, rr, i, _) in L], popped=None)
        records.append(rec)
        if not L:
            break
        v, rr, i, ch = L.pop(0)
        rec["popped"] = (v, rr, i)
        states = zoom(ch, max_active)
        r += 1
    return records


def run_bfs(subs, entries, states0, max_active, levels, width):
    """Breadth-first dynamic definition (the BFS-like query for dense
    outputs, Section 4.3): a landscape refined level by level.

    Readings where the paper gives only the strategy's name:

    * A node is one recursion: its 2^{#active} bins are reconstructed and its
      candidates are its ``width`` largest bins that still contain merged
      qubits, ordered by value descending, then bin index ascending.
    * Level 0 is the single node with the initial labels.  Level l + 1 has
      one node per each of the ``width`` best candidates over all level-l
      nodes, ordered by value descending, then parent node (in level order)
      ascending, then bin index ascending; the node zooms into its bin with
      the same rules as Algorithm 1 (the bin's active bits become fixed, the
      first ``max_active[c]`` merged qubits become active).
    * The query ends after ``levels`` levels or at a level with no
      candidates.

    Returns the nodes in level order: dict(level, parent (node index, -1
    for the root), parent_bin, states, bins, total, candidates [(value, bin)]).
    """
    nodes = []
    frontier = [(-1, 0, [st.copy() for st in states0])]
    for level in range(levels):
        if not frontier:
            break
        cands = []
        for parent, pbin, states in frontier:
            bins = bins_of(subs, entries, states)
            mine = []
            if any(st.merged for st in states):
                order = sorted(range(len(bins)), key=lambda i: (-bins[i], i))[:width]
                mine = [(float(bins[i]), i) for i in order]
            k = len(nodes)
            nodes.append(dict(level=level, parent=parent, parent_bin=pbin,
                              states=[st.copy() for st in states], bins=bins,
                              total=float(np.sum(bins)), candidates=mine))
            cands += [(v, k, i) for (v, i) in mine]
        cands.sort(key=lambda e: (-e[0], e[1], e[2]))
        frontier = [(k, i, zoom(child_states(nodes[k]["states"], i), max_active))
                    for (v, k, i) in cands[:width]]
    return nodes
