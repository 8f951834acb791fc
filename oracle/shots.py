"""Finite-shot emulation and the chi-square loss (test infrastructure only).

A QPU run reports the distribution of ``shots`` measured bit strings
(Section 2); here each row of a probability table (one subcircuit variant,
or one distribution) is sampled independently.  The oracle and the device
make every decision in integers, so they agree shot for shot:

* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC 2011) is the counter-based
  generator: key (seed low 32 bits, seed high 32 bits), counter (shot low,
  shot high, row low, row high); the shot's 64-bit uniform is
  word0 + 2^32 * word1 of the output.
* Probabilities are quantised to q_i = floor(min(max(p_i, 0), 1) * 2^52); the
  row's cumulative sums C_i = q_0 + ... + q_i are exact 64-bit integers.
* With T = C_last, a shot's target is t = floor(x * T / 2^64) in [0, T), and
  it lands on the first index i with C_i > t.  A row with T = 0 gets no
  counts.  The clamped entries of a row must sum below 2^12 so that C fits
  in 64 bits (a probability row sums to 1); the oracle rejects a row that
  does not.
* Frequencies are count / shots in FP64.

The chi-square loss of Eq. 3 sums (a_i - b_i)^2 / (a_i + b_i); terms with
a_i + b_i = 0 contribute 0 (the paper leaves 0/0 open).  It is applied as
written to reconstructed quasi-probabilities, whose negative entries can
make a term negative.
"""
from __future__ import annotations

import numpy as np

M32 = np.uint64(0xFFFFFFFF)
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on arrays of 32-bit counter words (held in uint64)
    with key words k0, k1.  Each round: the two products of counter words 0
    and 2 with the round multipliers split into high and low halves, the
    high halves xor-ed with the other counter words and the key; the key
    advances by the Weyl constants between rounds.

    Pinned by the published known-answer vectors of Philox4x32-10
    (tests/golden/philox4x32_10_kat.json)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & M32 for x in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for r in range(10):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & M32
        hi1, lo1 = p1 >> np.uint64(32), p1 & M32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & M32, lo1, (hi0 ^ c3 ^ k1) & M32, lo0
        if r < 9:
            k0 = (k0 + PHILOX_W0) & M32
            k1 = (k1 + PHILOX_W1) & M32
    return c0, c1, c2, c3


def mulhi64(x, T):
    """floor(x * T / 2^64) for uint64 arrays x and a uint64 scalar T."""
    x = np.asarray(x, dtype=np.uint64)
    T = np.uint64(T)
    s32 = np.uint64(32)
    xh, xl = x >> s32, x & M32
    th, tl = T >> s32, T & M32
    hh, hl, lh, ll = xh * th, xh * tl, xl * th, xl * tl
    mid = (hl & M32) + (lh & M32) + (ll >> s32)
    return hh + (hl >> s32) + (lh >> s32) + (mid >> s32)


def quantise(p):
    p = np.clip(np.asarray(p, dtype=np.float64), 0.0, 1.0)
    return np.floor(p * 2.0 ** 52).astype(np.uint64)


def shot_uniforms(seed, row, shots):
    s = np.arange(shots, dtype=np.uint64)
    w0, w1, _, _ = philox4x32_10(s & M32, s >> np.uint64(32), np.uint64(row & 0xFFFFFFFF),
                                 np.uint64(row >> 32), seed & 0xFFFFFFFF, seed >> 32)
    return w0 | (w1 << np.uint64(32))


def sample_counts(p_row, shots, seed, row):
    """Counts of one row's ``shots`` samples."""
    q = quantise(p_row)
    if float(np.sum(q.astype(np.float64))) >= 2.0 ** 64:
        raise ValueError("clamped row sum must be below 2^12")
    cdf = np.cumsum(q, dtype=np.uint64)
    counts = np.zeros(len(q), dtype=np.int64)
    T = int(cdf[-1]) if len(cdf) else 0
    if T == 0 or shots == 0:
        return counts
    t = mulhi64(shot_uniforms(seed, row, shots), T)
    idx = np.searchsorted(cdf, t, side="right")
    np.add.at(counts, idx, 1)
    return counts


def sample_frequencies(P, shots, seed):
    """Rows x cols probabilities -> empirical frequencies count / shots."""
    P = np.asarray(P, dtype=np.float64)
    flat = P.reshape(-1, P.shape[-1])
    out = np.zeros_like(flat)
    for r in range(flat.shape[0]):
        out[r] = sample_counts(flat[r], shots, seed, r) / float(shots)
    return out.reshape(P.shape)


def chi2(a, b):
    """Eq. 3 with 0/0 terms taken as 0."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    s = a + b
    nz = s != 0
    return float(np.sum((a[nz] - b[nz]) ** 2 / s[nz]))
