"""Pins of the finite-shot emulation and the chi-square loss (Eq. 3): integer
arithmetic against Python's exact integers, the generator's uniformity,
sampling against exact special cases and a goodness-of-fit bound, and the
loss against closed forms and its bounds."""
import json
import os

import numpy as np
import pytest

from oracle import attribution as at
from oracle import reconstruct as rc
from oracle import shots
from oracle import statevector as sv
from workloads import circuits as wc


def test_mulhi64_matches_exact_integers():
    rng = np.random.default_rng(1)
    x = rng.integers(0, 2 ** 63, size=2000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    for T in (1, 3, 2 ** 32 - 1, 2 ** 52, 2 ** 52 + 12345, 2 ** 63 + 5, 2 ** 64 - 1):
        got = shots.mulhi64(x, T)
        want = np.array([(int(v) * T) >> 64 for v in x], dtype=np.uint64)
        assert np.array_equal(got, want), T


def test_quantise_is_exact_floor():
    p = np.array([0.0, 1.0, 0.5, 1e-17, 2.0 ** -52, 0.1, 0.3333333333333333, -0.2, 1.5])
    q = shots.quantise(p)
    from fractions import Fraction
    for pi, qi in zip(p, q):
        c = min(max(Fraction(pi), 0), 1)
        assert int(qi) == (c * 2 ** 52).numerator // (c * 2 ** 52).denominator


def test_philox_known_answer_vectors():
    """The generator is Philox4x32-10 itself: the published known-answer
    vectors (tests/golden/philox4x32_10_kat.json) come out word for word."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")) as f:
        kat = json.load(f)["vectors"]
    assert len(kat) == 3
    for v in kat:
        c = [int(x, 16) for x in v["counter"]]
        k = [int(x, 16) for x in v["key"]]
        got = shots.philox4x32_10(*c, *k)
        assert ["%08x" % int(w) for w in got] == v["out"]


def test_generator_uniform_and_distinct():
    u = shots.shot_uniforms(seed=12345, row=3, shots=1 << 18)
    assert len(np.unique(u)) == len(u)
    top = (u >> np.uint64(56)).astype(np.int64)
    hist = np.bincount(top, minlength=256)
    e = len(u) / 256
    stat = float(np.sum((hist - e) ** 2 / e))
    assert stat < 255 + 6 * np.sqrt(2 * 255)          # 255 degrees of freedom, 6 sigma
    for b in range(64):
        ones = int(np.sum((u >> np.uint64(b)) & np.uint64(1)))
        assert abs(ones - len(u) / 2) < 6 * np.sqrt(len(u) / 4), b
    # rows and seeds give other streams
    assert not np.array_equal(u[:64], shots.shot_uniforms(12345, 4, 64))
    assert not np.array_equal(u[:64], shots.shot_uniforms(12346, 3, 64))


def test_sampling_special_cases():
    p = np.zeros(37)
    p[11] = 1.0
    c = shots.sample_counts(p, 5000, seed=7, row=0)
    assert c[11] == 5000 and c.sum() == 5000
    assert shots.sample_counts(np.zeros(9), 100, 7, 0).sum() == 0
    # negative entries count as zero probability
    p = np.array([-0.5, 0.0, 1.0, -1.0])
    assert shots.sample_counts(p, 300, 1, 2).tolist() == [0, 0, 300, 0]
    # same seed and row: same counts; frequencies are counts / shots
    P = np.random.default_rng(2).dirichlet(np.ones(64), size=3)
    f1 = shots.sample_frequencies(P, 1000, seed=9)
    f2 = shots.sample_frequencies(P, 1000, seed=9)
    assert np.array_equal(f1, f2)
    assert np.allclose(f1.sum(axis=1), 1.0)
    assert np.all(f1 * 1000 == np.round(f1 * 1000))
    # unnormalised rows are sampled in proportion; sums that overflow 64 bits
    # are rejected
    u = shots.sample_counts(np.array([0.5, 1.0, 1.0, 1.0]) * 1000, 10, 3, 0)
    assert u.sum() == 10
    with pytest.raises(ValueError):
        shots.sample_counts(np.ones(4096), 10, 3, 0)
    assert shots.sample_counts(np.ones(4095), 10, 3, 0).sum() == 10


def test_sampling_goodness_of_fit():
    rng = np.random.default_rng(3)
    p = rng.dirichlet(np.full(50, 2.0))
    n = 200000
    c = shots.sample_counts(p, n, seed=2024, row=5)
    e = n * p
    stat = float(np.sum((c - e) ** 2 / e))
    assert stat < 49 + 6 * np.sqrt(2 * 49)            # Pearson, 49 degrees of freedom


def test_chi2_closed_forms_and_bounds():
    a = np.array([0.5, 0.5, 0.0])
    assert shots.chi2(a, a) == 0.0
    b = np.array([0.25, 0.75, 0.0])   # the 0/0 term contributes nothing
    want = 0.25 ** 2 / 0.75 + 0.25 ** 2 / 1.25
    assert shots.chi2(a, b) == pytest.approx(want, rel=1e-15)
    assert shots.chi2(b, a) == pytest.approx(want, rel=1e-15)
    rng = np.random.default_rng(4)
    for _ in range(20):
        x, y = rng.dirichlet(np.ones(30)), rng.dirichlet(np.ones(30))
        tv2 = float(np.sum(np.abs(x - y)))
        assert 0.0 <= shots.chi2(x, y) <= tv2 <= 2.0
    # disjoint supports: every term is the full mass
    assert shots.chi2([1, 0], [0, 1]) == 2.0


def test_shot_noise_shrinks_with_shots_on_a_cut_circuit():
    """Sampled variants of the 8-qubit one-cut circuit, attributed and
    reconstructed, approach the state vector as the shots grow.  With few
    shots the reconstruction has negative entries, where Eq. 3's terms can be
    negative; the loss is compared in magnitude."""
    cc = wc.two_way_circuit_8q(seed=0)
    subs = cc.subcircuits()
    Vs = [sv.variant_probabilities(s) for s in subs]
    truth = sv.probabilities(cc.n_qubits, cc.ops)
    loss = []
    for n in (10000, 1000000):
        Vn = [shots.sample_frequencies(V, n, seed=11 + c) for c, V in enumerate(Vs)]
        E = [at.attribute(s, V) for s, V in zip(subs, Vn)]
        p = rc.apply_out_perm(rc.fd_definition(subs, E), cc.out_perm())
        loss.append(abs(shots.chi2(p, truth)))
    assert loss[1] < loss[0] / 10
