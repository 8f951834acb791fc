"""Synthetic subcircuit entry tensors and cut maps.

The paper's runtime study fed random numbers to the reconstructor instead of
subcircuit outputs (Section 5.4).  The workloads here follow that recipe:

* The identity-label row of every subcircuit (label 0, all cuts I) is a
  Dirichlet(0.1) draw over the subcircuit's 2^n output bins, made from
  normalised Gamma(0.1, 1) variates of numpy's PCG64 stream seeded with
  ``(seed, subcircuit)``.
* Every other row l is that row times U_l, where U_l[b] is uniform on
  [-1, 1) and comes from a counter-based generator: SplitMix64 (Steele,
  Lea & Flood, OOPSLA 2014) applied to ``counter ^ key``, with
  ``counter = l * 2^n + b`` and ``key = SplitMix64(seed << 32 | subcircuit)``;
  the top 53 bits of the hash give u in [0, 1) and U = 2u - 1.  Being
  counter-based, any single element can be regenerated on its own, which lets
  large tensors be filled on the device (``entries_torch``) and sampled
  columns be rebuilt on the host (``entries_columns``) with identical values.

Cut maps for chains of subcircuits are built here too (``chain_cutmap``):
subcircuit c measures the cuts of bond (c, c+1) and is initialised by those
of bond (c-1, c); cut ids are numbered bond by bond from the left.

Integer-valued entries (``integer_entries``) make every sum exact in binary
floating point, so index and layout errors show up as exact mismatches.
"""
from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1
_C0 = 0x9E3779B97F4A7C15
_C1 = 0xBF58476D1CE4E5B9
_C2 = 0x94D049BB133111EB


def _splitmix64_np(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z = x + np.uint64(_C0)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_C1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_C2)
        return z ^ (z >> np.uint64(31))


def _key(seed: int, sub: int) -> int:
    return int(_splitmix64_np(np.array([((seed & 0xFFFFFFFF) << 32) | (sub & 0xFFFFFFFF)],
                                       dtype=np.uint64))[0])


def uniform_pm1(seed: int, sub: int, counters: np.ndarray) -> np.ndarray:
    """U in [-1, 1) for the given counters (uint64 array), float64."""
    h = _splitmix64_np(counters.astype(np.uint64) ^ np.uint64(_key(seed, sub)))
    u = (h >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


def identity_row(seed: int, sub: int, n: int) -> np.ndarray:
    """Dirichlet(0.1) over 2^n bins (normalised Gamma variates)."""
    rng = np.random.default_rng([seed, sub])
    g = rng.gamma(0.1, 1.0, size=1 << n)
    return g / g.sum()


def dirichlet_entries(seed: int, sub: int, k: int, n: int) -> np.ndarray:
    """Full (4^k, 2^n) float64 entry tensor of subcircuit ``sub``."""
    row0 = identity_row(seed, sub, n)
    rows, cols = 4 ** k, 1 << n
    counters = np.arange(rows * cols, dtype=np.uint64)
    e = uniform_pm1(seed, sub, counters).reshape(rows, cols) * row0[None, :]
    e[0] = row0
    return e


def entries_columns(seed: int, sub: int, k: int, n: int, cols) -> np.ndarray:
    """Columns ``cols`` of ``dirichlet_entries(seed, sub, k, n)`` without
    building the whole tensor: shape (4^k, len(cols))."""
    cols = np.asarray(cols, dtype=np.uint64)
    row0 = identity_row(seed, sub, n)[cols.astype(np.int64)]
    rows = np.arange(4 ** k, dtype=np.uint64)
    counters = rows[:, None] * np.uint64(1 << n) + cols[None, :]
    e = uniform_pm1(seed, sub, counters.ravel()).reshape(counters.shape) * row0[None, :]
    e[0] = row0
    return e


def entries_torch(seed: int, sub: int, k: int, n: int, device, chunk_rows: int = 16):
    """Same tensor as ``dirichlet_entries`` built on ``device`` with torch
    integer ops (two's-complement int64 arithmetic wraps like uint64)."""
    import torch

    def s64(v):
        return v - (1 << 64) if v >= (1 << 63) else v

    rows, cols = 4 ** k, 1 << n
    row0 = torch.from_numpy(identity_row(seed, sub, n)).to(device)
    out = torch.empty((rows, cols), dtype=torch.float64, device=device)
    key = s64(_key(seed, sub))
    m53 = (1 << 53) - 1

    def lsr(z, s):
        return (z >> s) & ((1 << (64 - s)) - 1)

    col = torch.arange(cols, dtype=torch.int64, device=device)
    for r0 in range(0, rows, chunk_rows):
        r1 = min(rows, r0 + chunk_rows)
        rr = torch.arange(r0, r1, dtype=torch.int64, device=device)
        x = (rr[:, None] * cols + col[None, :]) ^ key
        z = x + s64(_C0)
        z = (z ^ lsr(z, 30)) * s64(_C1)
        z = (z ^ lsr(z, 27)) * s64(_C2)
        z = z ^ lsr(z, 31)
        u = (lsr(z, 11) & m53).to(torch.float64) * (2.0 ** -53)
        out[r0:r1] = (2.0 * u - 1.0) * row0[None, :]
        del x, z, u
    out[0] = row0
    return out


def integer_entries(rng: np.random.Generator, k: int, n: int, lo: int = -8, hi: int = 8):
    """Integer-valued (4^k, 2^n) float64 entries in [lo, hi]."""
    return rng.integers(lo, hi + 1, size=(4 ** k, 1 << n)).astype(np.float64)


def chain_cutmap(bonds, n_out):
    """Cut map of a chain of len(n_out) subcircuits.  ``bonds[c]`` cuts run
    from subcircuit c (measured) to c+1 (initialised).  Returns a list of
    (width, init_cut, meas_cut) per subcircuit.  Slots of subcircuit c: the
    init slots of the left bond (they are outputs), then the remaining
    outputs, then the measured slots of the right bond."""
    assert len(bonds) == len(n_out) - 1
    first = [0]
    for b in bonds:
        first.append(first[-1] + b)
    subs = []
    for c, n in enumerate(n_out):
        left = bonds[c - 1] if c > 0 else 0
        right = bonds[c] if c < len(bonds) else 0
        if left > n:
            raise ValueError("more arriving cuts than outputs")
        width = n + right
        init_cut = [-1] * width
        meas_cut = [-1] * width
        for j in range(left):
            init_cut[j] = first[c - 1] + j
        for j in range(right):
            meas_cut[n + j] = first[c] + j
        subs.append((width, init_cut, meas_cut))
    return subs


def chain_instance(seed: int, bonds, n_out):
    """Cut map + Dirichlet/uniform entries of a chain (host float64)."""
    cm = chain_cutmap(bonds, n_out)
    ks = [(bonds[c - 1] if c > 0 else 0) + (bonds[c] if c < len(bonds) else 0)
          for c in range(len(n_out))]
    ents = [dirichlet_entries(seed, c, ks[c], n_out[c]) for c in range(len(n_out))]
    return cm, ents


def chain_ks(bonds, n_sub):
    return [(bonds[c - 1] if c > 0 else 0) + (bonds[c] if c < len(bonds) else 0)
            for c in range(n_sub)]


def dd_batch_bonds(seed: int, n_inst: int = 16, n_sub: int = 4, k_range=(2, 6),
                   max_k_per_sub: int = 4):
    """Bond splits of a batch of chain instances: total cuts K uniform in
    k_range, then (k01, k12, ...) uniform over the splits of K with every
    subcircuit touching at most ``max_k_per_sub`` cuts.  A bond may carry 0
    cuts (then the chain falls apart into independent pieces there)."""
    rng = np.random.default_rng([seed, 0xDD])
    out = []
    for _ in range(n_inst):
        K = int(rng.integers(k_range[0], k_range[1] + 1))
        splits = []

        def rec(prefix, left):
            if len(prefix) == n_sub - 1:
                if left == 0:
                    splits.append(tuple(prefix))
                return
            for b in range(left + 1):
                rec(prefix + [b], left - b)
        rec([], K)
        ok = [s for s in splits if max(chain_ks(s, n_sub)) <= max_k_per_sub]
        out.append(ok[int(rng.integers(len(ok)))])
    return out
