"""GPU parity of the device state-vector simulator and subcircuit variants
against the oracle, through the C ABI, and the reconstruction of a 30-qubit
cut circuit against the device state vector of the uncut circuit.

Gates run in groups on LDS tiles (11 index bits, the 4 lowest always among
them; a group may take later gates that commute with the ones they
overtake), so the tests take circuits whose groups split on the tile width
and on the gate count per group (more than 40 gates), circuits narrower than
a tile, and slots that are both initialised and measured for cuts.  Values are sums of products of
unit-modulus-bounded factors: the bar is 1e-12 absolute against the oracle."""
import ctypes as C

import numpy as np
import pytest

from oracle import attribution as at
from oracle import cutmap
from oracle import reconstruct as rc
from oracle import statevector as sv
from workloads import circuits as wc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def cq():
    import paper_2205_05836_amd as m
    return m


def random_ops(rng, n, count, cz_frac=0.4):
    ops = []
    for _ in range(count):
        if n > 1 and rng.random() < cz_frac:
            a, b = rng.choice(n, size=2, replace=False)
            ops.append(wc.Op("cz", (int(a), int(b))))
        else:
            ops.append(wc.Op("u", (int(rng.integers(n)),), wc.haar_u2(rng)))
    return ops


@pytest.mark.parametrize("n,count,seed", [(1, 5, 0), (2, 12, 1), (5, 40, 2), (9, 80, 3), (10, 100, 4),
                                          (11, 120, 5), (14, 150, 6), (17, 60, 7)])
def test_random_circuits_match_oracle(n, count, seed):
    print(f"case n={n} gates={count} seed={seed}", flush=True)
    rng = np.random.default_rng(seed)
    ops = random_ops(rng, n, count)
    got = cq().cq_simulate_probabilities(n, ops).cpu().numpy()
    want = sv.probabilities(n, ops)
    assert np.max(np.abs(got - want)) < 1e-12
    assert abs(got.sum() - 1.0) < 1e-12


@pytest.mark.parametrize("n", [3, 11, 12])
def test_no_gates_gives_the_zero_state(n):
    """With no gates the probabilities are those of |0...0>: the first (here
    the only) pass generates that state instead of reading it."""
    got = cq().cq_simulate_probabilities(n, []).cpu().numpy()
    want = np.zeros(2 ** n)
    want[0] = 1.0
    assert np.array_equal(got, want)


def test_cz_runs_on_every_pair():
    """Runs of CZ gates on every pair of an 11-qubit register (one full
    tile): qubits 2-4 carry the most one-qubit gates of the first group (40
    gates), so the host puts them on the register bits (qubits 7-10, the
    lowest index bits, always sit on lane bits), and that group's CZ run
    opens with their three pairs; the runs hold pairs of two register bits,
    of a register bit and a thread-index bit, and of two thread-index bits,
    each folded into one sign per element."""
    rng = np.random.default_rng(9)
    n = 11
    layer = lambda: [wc.Op("u", (q,), wc.haar_u2(rng)) for q in range(n)]
    first = [(2, 3), (2, 4), (3, 4)]
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n) if (a, b) not in first]
    ops = [wc.Op("u", (q,), wc.haar_u2(rng)) for q in (2, 3, 4) for _ in range(3)] + layer()
    ops += [wc.Op("cz", pq) for pq in first] + [wc.Op("cz", pairs[i]) for i in rng.permutation(len(pairs))]
    pairs += first
    ops += layer() + [wc.Op("cz", pairs[i]) for i in rng.permutation(len(pairs))[:20]] + layer()
    got = cq().cq_simulate_probabilities(n, ops).cpu().numpy()
    assert np.max(np.abs(got - sv.probabilities(n, ops))) < 1e-12


def test_many_gates_on_few_qubits():
    """60 gates on 3 qubits of a 12-qubit register: groups split on the gate
    count, not on the tile width."""
    rng = np.random.default_rng(8)
    ops = random_ops(rng, 3, 60, cz_frac=0.3)
    ops = [wc.Op(o.name, tuple(q + 4 for q in o.qubits), o.matrix) for o in ops]
    ops += random_ops(rng, 12, 30)
    got = cq().cq_simulate_probabilities(12, ops).cpu().numpy()
    assert np.max(np.abs(got - sv.probabilities(12, ops))) < 1e-12


def _subcircuit_cases():
    cases = [("8q", wc.two_way_circuit_8q(0)), ("20q", wc.two_way_circuit_20q(1)),
             ("bv", wc.hidden_string_circuit([1, 0, 1, 1, 0, 1], [[0, 1, 2], [3, 4, 5]]))]
    seed = 900
    while len(cases) < 9:
        rng = np.random.default_rng(seed)
        seed += 1
        cc = wc.random_cut_circuit(rng, int(rng.integers(4, 9)), int(rng.integers(2, 4)),
                                   int(rng.integers(1, 5)), depth=5)
        if cc is not None and cc.cuts:
            cases.append((f"rand{seed - 1}", cc))
    return cases


@pytest.mark.parametrize("name,cc", _subcircuit_cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_variants_match_oracle(name, cc):
    print(f"variants {name}", flush=True)
    for spec in cc.subcircuits():
        got = cq().cq_variant_probabilities(spec).cpu().numpy()
        want = sv.variant_probabilities(spec)
        assert got.shape == want.shape
        assert np.max(np.abs(got - want)) < 1e-12
        assert np.allclose(got.sum(axis=-1), 1.0, atol=1e-12)


@pytest.mark.parametrize("w,init,meas", [(13, (0, 6), (3, 9)), (11, (0, 6), (10,)), (12, (0, 6), ()),
                                         (12, (5,), (2, 11))])
def test_variants_bases_in_one_pass(w, init, meas):
    """A register of at least 11 slots with at most two measured cut ends:
    one pass writes every measurement basis (up to nine).  With one or two
    initialised ends only the 2^r computational init strings are simulated
    and each of the 4^r init strings is combined from them in that pass."""
    rng = np.random.default_rng(40 + w + len(init))
    ic = [-1] * w
    mc = [-1] * w
    for i, s_ in enumerate(init):
        ic[s_] = i
    for i, s_ in enumerate(meas):
        mc[s_] = len(init) + i
    ops = random_ops(rng, w, 6 * w)
    spec = wc.SubcircuitSpec(w, ic, mc, [(q, 0) for q in range(w)], ops)
    got = cq().cq_variant_probabilities(spec).cpu().numpy()
    want = sv.variant_probabilities(spec)
    assert got.shape == want.shape == (4 ** len(init), 3 ** len(meas), 2 ** w)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("states", [1, 3])
def test_variants_with_a_smaller_workspace(states):
    """A workspace of `states` states (fewer than the 16 the size query asks
    for): the initial states run in batches of that many, the last one
    partial, with the same results."""
    from paper_2205_05836_amd import _lib
    from paper_2205_05836_amd.api import _Subs, _dev_ptr, _gates, _stream
    rng = np.random.default_rng(77)
    w = 12
    ic = [-1] * w
    mc = [-1] * w
    ic[1], ic[7], mc[4], mc[10] = 0, 1, 2, 3
    ops = random_ops(rng, w, 5 * w)
    spec = wc.SubcircuitSpec(w, ic, mc, [(q, 0) for q in range(w)], ops)
    out = torch.full((16, 9, 2 ** w), -1.0, dtype=torch.float64, device=DEV)
    nbytes = states * (16 << w)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=DEV)
    subs = _Subs([spec])
    arr, cnt = _gates(ops)
    assert _lib.lib().cq_variant_probabilities(subs.ptr(), arr, cnt, _dev_ptr(out), _dev_ptr(ws), nbytes,
                                               _stream(None)) == 0
    torch.cuda.synchronize()
    want = sv.variant_probabilities(spec)
    assert np.max(np.abs(out.cpu().numpy() - want)) < 1e-12


def test_slot_both_initialised_and_measured():
    """A wire cut twice leaves a middle segment that a cut initialises and
    another cut measures: init and basis digits both land on one slot."""
    seed, found = 950, 0
    while found < 2 and seed < 1200:
        rng = np.random.default_rng(seed)
        seed += 1
        cc = wc.random_cut_circuit(rng, 5, 2, 4, depth=6)
        if cc is None:
            continue
        for spec in cc.subcircuits():
            both = [s for s in range(spec.width) if spec.init_cut[s] != -1 and spec.meas_cut[s] != -1]
            if both:
                found += 1
                got = cq().cq_variant_probabilities(spec).cpu().numpy()
                assert np.max(np.abs(got - sv.variant_probabilities(spec))) < 1e-12
    assert found >= 1


def _restrict(ops, qubits):
    index = {q: i for i, q in enumerate(qubits)}
    return [wc.Op(o.name, tuple(index[q] for q in o.qubits), o.matrix) for o in ops
            if all(q in index for q in o.qubits)]


def test_30_qubit_product_circuit_against_oracle_halves():
    """A 30-qubit brickwork whose two halves never interact (the CZ across
    the middle is masked out): the device distribution must be the outer
    product of the oracle's two 15-qubit distributions."""
    cc = wc.masked_brickwork(30, 6, [], lambda q, s: 0 if q < 15 else 1, seed=12)
    assert not any(o.name == "cz" and min(o.qubits) < 15 <= max(o.qubits) for o in cc.ops)
    print("30q product circuit", flush=True)
    p = cq().cq_simulate_probabilities(30, cc.ops)
    pa = sv.probabilities(15, _restrict(cc.ops, range(15)))
    pb = sv.probabilities(15, _restrict(cc.ops, range(15, 30)))
    ref = torch.outer(torch.from_numpy(pa).to(DEV), torch.from_numpy(pb).to(DEV)).reshape(-1)
    err = torch.max(torch.abs(p - ref)).item()
    assert err <= 1e-13 * torch.max(ref).item()
    assert abs(torch.sum(p).item() - 1.0) < 1e-10


def test_32_qubit_product_circuit_sampled_against_oracle_halves():
    """32 qubits (2^32 amplitudes, indices past 2^31 and 2^21 tiles): two
    non-interacting 16-qubit halves, 10^6 sampled probabilities against the
    products of the oracle's half distributions."""
    cc = wc.masked_brickwork(32, 4, [], lambda q, s: 0 if q < 16 else 1, seed=13)
    print("32q product circuit", flush=True)
    p = cq().cq_simulate_probabilities(32, cc.ops)
    pa = sv.probabilities(16, _restrict(cc.ops, range(16)))
    pb = sv.probabilities(16, _restrict(cc.ops, range(16, 32)))
    idx = np.random.default_rng(14).integers(0, 1 << 32, size=1000000, dtype=np.int64)
    idx[:4] = [0, (1 << 32) - 1, (1 << 31), (1 << 31) - 1]
    got = p[torch.from_numpy(idx).to(DEV)].cpu().numpy()
    total = torch.sum(p).item()
    del p
    want = pa[idx >> 16] * pb[idx & 0xFFFF]
    assert np.max(np.abs(got - want)) <= 1e-13 * max(pa.max() * pb.max(), 1e-300)
    assert abs(total - 1.0) < 1e-10


def test_30_qubit_cut_circuit_reconstruction_matches_state_vector():
    """The 30-qubit two-way cut circuit (subcircuits of 16 and 18 slots, four
    cuts): device variants, attribution and FP64 full definition against the
    device state vector of the uncut circuit, two code paths that share no
    kernels."""
    m = cq()
    cc = wc.two_way_circuit_30q()
    subs = cc.subcircuits()
    print("30q variants", flush=True)
    E = [m.cq_attribute(s, m.cq_variant_probabilities(s)) for s in subs]
    p = m.cq_reconstruct_fd(subs, E, prec="fp64", out_perm=cc.out_perm())
    del E
    print("30q state vector", flush=True)
    truth = m.cq_simulate_probabilities(30, cc.ops)
    torch.cuda.synchronize()
    d = torch.abs(p - truth)
    assert torch.max(d).item() <= 1e-12 * torch.max(truth).item()
    assert 0.5 * torch.sum(d).item() < 1e-10
    assert abs(torch.sum(truth).item() - 1.0) < 1e-10
    assert torch.min(truth).item() >= 0.0


def test_state_vector_arguments_rejected_before_launch():
    from paper_2205_05836_amd import _lib
    from paper_2205_05836_amd.api import _dev_ptr, _gates, _stream
    L = _lib.lib()
    out = torch.full((16,), -2.0, dtype=torch.float64, device=DEV)
    ws = torch.empty(16 * 16, dtype=torch.uint8, device=DEV)
    good, _ = _gates([("u", 0, np.eye(2))])
    cases = [(0, [], -2), (35, [], -2), (4, [("u", 4, np.eye(2))], -1), (4, [("cz", 1, 1)], -1),
             (4, [("cz", 0, 7)], -1), (4, [("u", 0, np.array([[np.nan, 0], [0, 1]]))], -1)]
    for n, ops, code in cases:
        arr, cnt = _gates(ops)
        assert L.cq_simulate_probabilities(n, arr, cnt, _dev_ptr(out), _dev_ptr(ws), 256, _stream(None)) == code
    bad_kind, _ = _gates([("u", 0, np.eye(2))])
    bad_kind[0].kind = 5
    assert L.cq_simulate_probabilities(4, bad_kind, 1, _dev_ptr(out), _dev_ptr(ws), 256, _stream(None)) == -1
    assert L.cq_simulate_probabilities(4, good, 1, _dev_ptr(out), _dev_ptr(ws), 255, _stream(None)) == -5
    torch.cuda.synchronize()
    assert torch.all(out == -2.0)
    with pytest.raises(cq().CQError):
        cq().cq_variant_probabilities((3, [0, -1, -1], [-1, -1, 0]), [])


def test_found_cuts_reconstruct_on_device():
    """An 8-qubit circuit cut by the library's exact search for 5-qubit
    devices, then run end to end on the device (variants, attribution, FP64
    full definition) against the oracle's state vector of the uncut
    circuit."""
    m = cq()
    rng = np.random.default_rng(31)
    n, ops = 8, []
    for t in range(3):
        ops += [wc.Op("u", (q,), wc.haar_u2(rng)) for q in range(n)]
        ops += [wc.Op("cz", (i, i + 1)) for i in range(t % 2, n - 1, 2)]
    ops += [wc.Op("u", (q,), wc.haar_u2(rng)) for q in range(n)]
    found = m.cq_find_cuts(n, ops, max_width=5, max_subcircuits=3)
    # subcircuits are numbered 0.. in order of first use, with none skipped
    assert sorted(set(found["cluster"])) == list(range(found["n_subcircuits"]))
    cc = wc.cut_circuit_from_clusters(n, ops, found["cluster"])
    subs = cc.subcircuits()
    assert found["n_cuts"] >= 1 and max(s.width for s in subs) <= 5
    # the search cuts one wire twice here, so some slot is initialised by one
    # cut and measured for another: attribution's mixed-slot case runs
    assert any(i >= 0 and mc >= 0 for s in subs for i, mc in zip(s.init_cut, s.meas_cut))
    E = [m.cq_attribute(s, m.cq_variant_probabilities(s)) for s in subs]
    p = m.cq_reconstruct_fd(subs, E, prec="fp64", out_perm=cc.out_perm()).cpu().numpy()
    assert np.max(np.abs(p - sv.probabilities(n, ops))) < 1e-12
