"""Exhaustive cut search for tiny circuits (test infrastructure only).

Section 4.1: the two-qubit gates are the vertices of the circuit's DAG and
the qubit wires between consecutive two-qubit gates are its edges; a
clustering of the vertices into subcircuits cuts the edges between
clusters.  The objective is the multiplication count L of Section 4.1,

    L = 4^K * sum_{c=2}^{n_C} prod_{i=1}^{c} 2^{n_i},

read with n_i = the outputs of subcircuit i (the length log2 of its entry
vectors in Eq. 1) and the subcircuits ordered by n_i ascending; L = 0 when
there is no cut.  A subcircuit's width (the qubits a device must hold) is
the number of wire segments it contains.
"""
from __future__ import annotations

import itertools


def structure(n_qubits, gates, labels):
    """(K, widths, outputs) of a clustering: labels[g] is gate g's cluster."""
    n_sub = max(labels) + 1
    width = [0] * n_sub
    measured = [0] * n_sub
    cuts = 0
    for q in range(n_qubits):
        on_q = [g for g, pair in enumerate(gates) if q in pair]
        if not on_q:
            raise ValueError(f"qubit {q} takes part in no two-qubit gate")
        width[labels[on_q[0]]] += 1          # the wire's first segment
        for a, b in zip(on_q, on_q[1:]):
            if labels[a] != labels[b]:       # a cut between consecutive gates
                cuts += 1
                measured[labels[a]] += 1
                width[labels[b]] += 1
    outputs = [w - m for w, m in zip(width, measured)]
    return cuts, width, outputs


def cost(cuts, outputs):
    if len(outputs) < 2:
        return 0.0
    n = sorted(outputs)
    total, prod = 0, 2 ** n[0]
    for c in range(1, len(n)):
        prod *= 2 ** n[c]
        total += prod
    return float(4 ** cuts * total)


def canonical(labels):
    """Relabel clusters in order of first use."""
    seen = {}
    return tuple(seen.setdefault(x, len(seen)) for x in labels)


def best_clustering(n_qubits, gates, max_width, max_subcircuits):
    """Minimum-L clustering over all label assignments; ties go to the
    lexicographically smallest canonical label string.  Returns None when
    nothing fits."""
    best = None
    for raw in itertools.product(range(max_subcircuits), repeat=len(gates)):
        labels = canonical(raw)
        if labels != raw:
            continue
        cuts, width, outputs = structure(n_qubits, gates, labels)
        if max(width) > max_width:
            continue
        L = cost(cuts, outputs)
        key = (L, labels)
        if best is None or key < best[0]:
            best = (key, cuts, max(labels) + 1)
    if best is None:
        return None
    (L, labels), cuts, n_sub = best
    return dict(cluster=list(labels), cost=L, n_cuts=cuts, n_subcircuits=n_sub)
