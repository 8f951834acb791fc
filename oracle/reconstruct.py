"""Eq. 1, the Kronecker-sum reconstruction.  Test infrastructure only.

    P = 2^-K  sum over all 4^K labelings l of the K cuts of
              kron_{c = 0 .. n_C-1} E_c[l restricted to c's cuts]

Eq. 1 prints the sum without the factor; the 1/2 per cut of the Pauli
decomposition (see ``attribution``) is applied here, once.  Output order:
subcircuit 0's outputs are the most significant bits; ``apply_out_perm``
maps that concatenated order to the uncut circuit's qubit order.

Three forms of the same sum:

* ``fd_definition`` -- the sum over labelings as written, one Kronecker
  product per labeling (small n only).
* ``fd_per_bin``    -- the same sum evaluated for chosen output bins only.
* ``fd_contract``   -- the same sum handed to numpy.einsum, which contracts
  the shared label indices pairwise with BLAS (used for larger cases and as
  the timed CPU baseline).
"""
from __future__ import annotations

import itertools
import string

import numpy as np

from . import cutmap


def fd_definition(subs, entries):
    K = cutmap.total_cuts(subs)
    n = sum(len(cutmap.outputs(s)) for s in subs)
    p = np.zeros(2 ** n)
    for labels in itertools.product(range(4), repeat=K):
        v = np.ones(1)
        for s, E in zip(subs, entries):
            v = np.kron(v, E[cutmap.local_label(s, labels)])
        p += v
    return p * 2.0 ** -K


def apply_out_perm(p, perm):
    """Reorder a concatenated-order vector so that bit position q (most
    significant first) of the result holds uncut qubit q; ``perm[i]`` is the
    qubit carried by concatenated bit i."""
    n = len(perm)
    t = np.asarray(p).reshape((2,) * n)
    axes = [0] * n
    for i, q in enumerate(perm):
        axes[q] = i
    return np.transpose(t, axes).reshape(-1)


def _split_bins(subs, bins):
    ns = [len(cutmap.outputs(s)) for s in subs]
    bins = np.asarray(bins, dtype=np.int64)
    parts, shift = [], sum(ns)
    for n in ns:
        shift -= n
        parts.append((bins >> shift) & ((1 << n) - 1))
    return parts


def _einsum_terms(subs):
    """einsum subscripts: one letter per cut, one per subcircuit output axis."""
    letters = iter(string.ascii_letters)
    K = cutmap.total_cuts(subs)
    cut_letter = [next(letters) for _ in range(K)]
    out_letter = [next(letters) for _ in subs]
    terms = []
    for c, s in enumerate(subs):
        terms.append("".join(cut_letter[x] for x in cutmap.incident_cuts(s)) + out_letter[c])
    return terms, out_letter, K


def fd_per_bin(subs, entries, bins):
    """p at the given concatenated-order output bins."""
    parts = _split_bins(subs, bins)
    terms, _, K = _einsum_terms(subs)
    ops, sub_terms = [], []
    for s, E, b, t in zip(subs, entries, parts, terms):
        k = len(cutmap.incident_cuts(s))
        cols = np.asarray(E)[:, b]                      # (4^k, nbins)
        ops.append(cols.reshape((4,) * k + (len(b),)))
        sub_terms.append(t[:-1] + "Z")
    expr = ",".join(sub_terms) + "->Z"
    return np.einsum(expr, *ops, optimize=True) * 2.0 ** -K


def fd_contract(subs, entries, lead=None):
    """Full p in concatenated order.  ``lead=(start, stop)`` restricts
    subcircuit 0's output index to that range (the result then covers only
    those leading bits)."""
    terms, out_letter, K = _einsum_terms(subs)
    ops = []
    for c, (s, E) in enumerate(zip(subs, entries)):
        k = len(cutmap.incident_cuts(s))
        E = np.asarray(E)
        if c == 0 and lead is not None:
            E = E[:, lead[0]:lead[1]]
        ops.append(E.reshape((4,) * k + (E.shape[1],)))
    expr = ",".join(terms) + "->" + "".join(out_letter)
    return np.einsum(expr, *ops, optimize=True).reshape(-1) * 2.0 ** -K
