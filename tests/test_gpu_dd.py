"""GPU parity of dynamic definition (Algorithm 1) against the oracle, through
the C ABI: per recursion the labels (active / merged / fixed masks and fixed
values), the bins, the FP64 total, the list L after the update and the pop.

Integer-valued entries make every bin exact, so there bins, list values and
the zoom path must match bit for bit; on Dirichlet/uniform data the FP64 path
must match within 1e-10 and take the same zoom path."""
import numpy as np
import pytest

from oracle import attribution as at
from oracle import cutmap
from oracle import dd
from oracle import statevector as sv
from workloads import circuits as wc
from workloads import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def cq():
    import paper_2205_05836_amd as m
    return m


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def mask(positions):
    m = 0
    for p in positions:
        m |= 1 << int(p)
    return m


def instance(cm, E, states, max_active):
    return dict(subs=cm, entries=[to_dev(e) for e in E],
                active=[mask(s.active) for s in states], merged=[mask(s.merged) for s in states],
                fixed=[mask(s.fixed.keys()) for s in states],
                fixed_vals=[mask(p for p, v in s.fixed.items() if v) for s in states],
                max_active=list(max_active))


def max_bins_log2(cm, states, max_active):
    ns = [len(cutmap.outputs(s)) for s in cm]
    return sum(max(len(s.active), min(m, n)) for s, m, n in zip(states, max_active, ns))


def run_gpu(cm, E, states, max_active, R, prec, launch="graph"):
    A = max_bins_log2(cm, states, max_active)
    dt = torch.float64 if prec == "fp64" else torch.float32
    bins = [torch.full((2 ** A,), float("nan"), dtype=dt, device=DEV) for _ in range(R)]
    recs, done = cq().cq_reconstruct_dd([instance(cm, E, states, max_active)], prec, R, bins=bins,
                                        launch=launch)
    torch.cuda.synchronize()
    return recs[0], done[0], bins


def _unique_positions(vals, gap):
    """Positions of a sorted list whose value is separated from both
    neighbours by more than `gap` (their rank does not depend on rounding)."""
    out = []
    for i, v in enumerate(vals):
        lo = i == 0 or abs(vals[i - 1] - v) > gap
        hi = i == len(vals) - 1 or abs(vals[i + 1] - v) > gap
        if lo and hi:
            out.append(i)
    return out


TILE_KEYS = ("tiles", "tiles_run")


def strip_tiles(recs):
    """Records without the tile counts (which only the fused path reports)."""
    return [[{k: v for k, v in r.items() if k not in TILE_KEYS} for r in rr] for rr in recs]


def check_tile_counts(fused, stored):
    """The stored path reports no tiles.  The fused path's selecting step
    covers the recursion's 2^n_active bins with 128 x 128 tiles (so between
    2^n_active / 2^14 and 2^n_active of them) whenever the recursion has
    merged outputs, and evaluates each at most once besides the warm-up tiles
    (at most 64)."""
    for rf, rs in zip(fused, stored):
        for a, b in zip(rf, rs):
            assert b["tiles"] == 0 and b["tiles_run"] == 0
            t, bins = a["tiles"], 2 ** a["n_active"]
            if not any(a["merged"]):
                assert t == 0 and a["tiles_run"] == 0
                continue
            assert -(-bins // 2 ** 14) <= t <= bins, (t, bins)
            assert 1 <= a["tiles_run"] <= t + min(t, 64), (a["tiles_run"], t)


def compare(cm, E, states, max_active, R, prec, tol, launch="graph"):
    """Walks the recursions of both runs.  Labels, bins and list values must
    agree; list identities must agree wherever the order is fixed by values
    more than `gap` apart (ties up to rounding may rank either way, Algorithm 1
    admits both); the comparison stops after a pop that was such a tie, since
    both zoom paths are then correct."""
    ref = dd.run(cm, E, states, max_active, R)
    got, done, bins = run_gpu(cm, E, states, max_active, R, prec, launch)
    gap = 0.0 if tol == 0 else 1e-10
    for r, (g, o) in enumerate(zip(got, ref)):
        st = o["states"]
        assert g["active"] == [mask(s.active) for s in st], r
        assert g["merged"] == [mask(s.merged) for s in st], r
        assert g["fixed"] == [mask(s.fixed.keys()) for s in st], r
        assert g["fixed_vals"] == [mask(p for p, v in s.fixed.items() if v) for s in st], r
        nb = o["bins"].size
        assert g["n_active"] == int(np.log2(nb))
        b = bins[r][:nb].cpu().numpy().astype(np.float64)
        if tol == 0:
            assert np.array_equal(b, o["bins"]), r
            assert g["total"] == o["bins"].sum()
        else:
            assert np.max(np.abs(b - o["bins"])) < tol, r
            assert abs(g["total"] - o["bins"].sum()) < 1e-10
        gv = [v for (v, _, _) in g["list"]]
        ov = [v for (v, _, _) in o["L"]]
        assert len(gv) == len(ov), r
        assert all(abs(a - c) <= gap for a, c in zip(gv, ov)), r
        if tol == 0:
            # exact arithmetic: ties are broken by (recursion, bin index) on both sides
            assert [e[1:] for e in g["list"]] == [e[1:] for e in o["L"]], r
        for i in _unique_positions(ov, 2 * gap):
            assert g["list"][i][1:] == o["L"][i][1:], (r, i)
        assert g["popped"] == (o["popped"] is not None)
        if o["popped"] is None:
            assert done == r + 1 == len(ref)
            return
        if tol != 0 and 0 not in _unique_positions(ov, 2 * gap):
            return  # tied pop: both continuations are valid
    assert done == len(ref)


@pytest.mark.parametrize("launch", ["graph", "direct"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(4))
def test_integer_entries_exact(case, prec, launch):
    rng = np.random.default_rng(50 + case)
    bonds = [[1, 1], [2, 1], [0, 2], [1, 2, 1]][case]
    ns = [[4, 4, 4], [5, 3, 6], [3, 4, 5], [3, 3, 4, 3]][case]
    cm = syn.chain_cutmap(bonds, ns)
    E = [syn.integer_entries(rng, k, n, lo=-3, hi=6) for k, n in zip(syn.chain_ks(bonds, len(ns)), ns)]
    M = [1 + (case % 2)] * len(ns)
    print(f"dd int case {case} {prec} {launch}", flush=True)
    compare(cm, E, dd.initial_states(cm, M), M, R=4, prec=prec, tol=0, launch=launch)


def test_physical_circuit_fp64():
    cc = wc.two_way_circuit_8q(0)
    subs = cc.subcircuits()
    E = [at.attribute(s, sv.variant_probabilities(s)) for s in subs]
    M = [2, 1]
    compare(subs, E, dd.initial_states(subs, M), M, R=5, prec="fp64", tol=1e-12)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-6), ("bf16_split", 1e-6),
                                      ("fp16_split", 1e-6), ("fp16", 1e-3), ("bf16", 2e-2)])
def test_dirichlet_chain(prec, tol):
    cm, E = syn.chain_instance(61, [2, 2], [7, 6, 7])
    M = [2, 2, 2]
    compare(cm, E, dd.initial_states(cm, M), M, R=4, prec=prec, tol=tol)


LABEL_SHIFT = {0: 0, 1: 20, 2: -20, 3: 10}   # digit I, X, Y, Z -> log2 factor


def imbalance_labels(cm, E, shift=LABEL_SHIFT):
    """Rows scaled per cut label: digit d at cut j gets 2^shift[d] on the
    subcircuit measuring j and 2^-shift[d] on the one initialising it, so
    every labelling term of Eq. 1 -- hence every bin -- keeps its value
    exactly, while label rows within a subcircuit differ by up to 2^80."""
    out = []
    for sub, e in zip(cm, E):
        _, init, meas = sub
        cuts = cutmap.incident_cuts(sub)
        k = len(cuts)
        ex = np.zeros(4 ** k, dtype=np.int64)
        for l in range(4 ** k):
            for p, cut in enumerate(cuts):
                d = (l >> (2 * (k - 1 - p))) & 3
                ex[l] += shift[d] if cut in meas else -shift[d]
        out.append(np.ldexp(e, ex[:, None]))
    return out


@pytest.mark.parametrize("prec,tol", [("fp16_split", 1e-6), ("fp16", 1e-3)])
def test_label_balance_on_imbalanced_labels(prec, tol):
    """Dynamic definition in FP16 on label rows 2^+-20 apart per digit: with
    the per-label balance of the reduced entries every recursion matches the
    oracle as on balanced input; without it the FP16 operands overflow or
    lose the small rows.  The fused top-C path (no bins stored) gives the
    same records as the stored-bin path."""
    m = cq()
    cm, E = syn.chain_instance(61, [2, 2], [7, 6, 7])
    Ei = imbalance_labels(cm, E)
    M = [2, 2, 2]
    st = dd.initial_states(cm, M)
    try:
        m.cq_label_balance_enable(1)
        compare(cm, Ei, st, M, R=4, prec=prec, tol=tol)
        stored, done_s, _ = run_gpu(cm, Ei, st, M, 4, prec)
        fused, done_f = m.cq_reconstruct_dd([instance(cm, Ei, st, M)], prec, 4)
        torch.cuda.synchronize()
        m.cq_label_balance_enable(0)
        _, _, bins_off = run_gpu(cm, Ei, st, M, 1, prec)
    finally:
        m.cq_label_balance_enable(1)
    assert done_f[0] == done_s
    assert strip_tiles(fused) == strip_tiles([stored])
    ref = dd.run(cm, Ei, st, M, 1)
    nb = ref[0]["bins"].size
    err_off = np.max(np.abs(bins_off[0][:nb].cpu().numpy().astype(np.float64) - ref[0]["bins"]))
    print(f"{prec}: recursion-0 bins without the balance, max abs err {err_off:.3e}", flush=True)
    assert not err_off < tol  # overflowing operands give inf or nan, which also counts


COL_SHIFT = [0, 12, 10]   # per subcircuit: column b scaled by 2^(-shift * popcount(b))


def imbalance_columns(E, shift=COL_SHIFT):
    """Columns (output bit patterns) scaled down by 2^-shift per set bit:
    recursion-0 bins then span about 2^-40 of each other, far below FP16's
    range once converted without a per-column scale."""
    out = []
    for s, e in zip(shift, E):
        pc = np.array([bin(b).count("1") for b in range(e.shape[1])], dtype=np.int64)
        out.append(np.ldexp(e, -s * pc[None, :]))
    return out


@pytest.mark.parametrize("prec,tol", [("fp16_split", 1e-5), ("fp16", 2e-3)])
def test_column_scaling_on_imbalanced_columns(prec, tol):
    """Dynamic definition in FP16 with output columns 2^-10 .. 2^-12 apart
    per set bit (on top of imbalanced label rows): the column scaling of the
    reduced entries keeps every recursion-0 bin accurate relative to its own
    magnitude (the bins of |E|, which bound every term), tiny bins included;
    the fused top-C path, whose tile bounds carry the exponents, gives the
    same records as the stored-bin path."""
    m = cq()
    cm, E = syn.chain_instance(64, [2, 2], [7, 6, 7])
    Ei = imbalance_columns(imbalance_labels(cm, E))
    M = [2, 2, 2]
    st = dd.initial_states(cm, M)
    compare(cm, Ei, st, M, R=4, prec=prec, tol=tol)
    stored, done_s, bins = run_gpu(cm, Ei, st, M, 4, prec)
    fused, done_f = m.cq_reconstruct_dd([instance(cm, Ei, st, M)], prec, 4)
    torch.cuda.synchronize()
    try:
        m.cq_column_scaling_enable(False)
        _, _, bins_off = run_gpu(cm, Ei, st, M, 1, prec)
    finally:
        m.cq_column_scaling_enable(True)
    assert done_f[0] == done_s
    assert strip_tiles(fused) == strip_tiles([stored])
    ref = dd.run(cm, Ei, st, M, 1)[0]["bins"]
    scale = dd.run(cm, [np.abs(e) for e in Ei], st, M, 1)[0]["bins"]
    assert scale.min() < 2.0 ** -30 * scale.max()   # the bins really span FP16's range

    def rel_err(b):
        got = b[0][:ref.size].cpu().numpy().astype(np.float64)
        return np.max(np.abs(got - ref) / scale)

    rel, rel_off = rel_err(bins), rel_err(bins_off)
    print(f"{prec}: recursion-0 bins, max error relative to |E| bins {rel:.3e}, "
          f"without column scaling {rel_off:.3e}", flush=True)
    assert rel < tol
    assert not rel_off < tol   # the small bins are lost (or nan) without it


def test_initial_fixed_bits_and_single_recursion():
    cm, E = syn.chain_instance(62, [1, 2], [5, 5, 5])
    states = [dd.SubState([0], [2, 3, 4], {1: 1}), dd.SubState([], [0, 1, 2, 3, 4], {}),
              dd.SubState([4, 1], [0], {2: 0, 3: 1})]
    compare(cm, E, states, [2, 1, 1], R=1, prec="fp64", tol=1e-10)
    compare(cm, E, states, [2, 1, 1], R=6, prec="fp64", tol=1e-10)


def test_all_merged_gives_one_bin():
    cm, E = syn.chain_instance(63, [2, 1], [4, 4, 4])
    states = [dd.SubState([], [0, 1, 2, 3], {}) for _ in range(3)]
    compare(cm, E, states, [1, 1, 1], R=3, prec="fp64", tol=1e-10)


def test_batch_of_instances_matches_one_by_one():
    m = cq()
    insts, refs = [], []
    for i, (bonds, ns) in enumerate([([1, 1], [4, 4, 4]), ([2, 0, 1], [3, 4, 3, 4])]):
        cm, E = syn.chain_instance(70 + i, bonds, ns)
        M = [2] * len(ns)
        st = dd.initial_states(cm, M)
        insts.append(instance(cm, E, st, M))
        refs.append(dd.run(cm, E, st, M, 3))
    recs, done = m.cq_reconstruct_dd(insts, "fp64", 3)
    for g, o, d in zip(recs, refs, done):
        assert d == len(o)
        for gr, orr in zip(g, o):
            assert abs(gr["total"] - orr["bins"].sum()) < 1e-10
            assert [(rr, i) for (_, rr, i) in gr["list"]] == [(rr, i) for (_, rr, i) in orr["L"]]


def test_hidden_string_found():
    secret = [1, 1, 0, 1, 0, 0, 1, 1, 0, 1]
    groups = [[0, 1, 2], [3, 4, 5, 6], [7, 8, 9]]
    cc = wc.hidden_string_circuit(secret, groups)
    subs = cc.subcircuits()
    E = [at.attribute(s, sv.variant_probabilities(s)) for s in subs]
    M = [1, 1, 1]
    R = 5
    got, done, bins = run_gpu(subs, E, dd.initial_states(subs, M), M, R, "fp64")
    # the first recursion with nothing merged resolves every qubit: one bin holds p = 1
    full = [r for r, g in enumerate(got) if all(m == 0 for m in g["merged"])]
    assert full
    r = full[0]
    nb = 2 ** got[r]["n_active"]
    assert bins[r][:nb].cpu().numpy().max() == pytest.approx(1.0, abs=1e-12)
    compare(subs, E, dd.initial_states(subs, M), M, R, "fp64", 1e-12)


def test_graph_and_direct_launches_agree():
    """The captured graph replays exactly the launches of the direct mode."""
    m = cq()
    insts = []
    for i, (bonds, ns) in enumerate([([2, 1], [5, 6, 4]), ([1, 1, 1], [4, 3, 4, 3])]):
        cm, E = syn.chain_instance(90 + i, bonds, ns)
        M = [2] * len(ns)
        insts.append(instance(cm, E, dd.initial_states(cm, M), M))
    R = 4
    out = {}
    for launch in ("graph", "direct"):
        bins = []
        for inst in insts:
            A = max_bins_log2(inst["subs"], dd.initial_states(inst["subs"], inst["max_active"]),
                              inst["max_active"])
            bins += [torch.full((2 ** A,), float("nan"), dtype=torch.float32, device=DEV) for _ in range(R)]
        recs, done = m.cq_reconstruct_dd(insts, "fp32", R, bins=bins, launch=launch)
        out[launch] = (recs, done, [b.cpu().numpy() for b in bins])
    (rg, dg, bg), (rd, ddn, bd) = out["graph"], out["direct"]
    assert dg == ddn
    assert rg == rd
    for x, y in zip(bg, bd):
        assert np.array_equal(x, y, equal_nan=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16_split"])
def test_fused_top_c_matches_stored_bins(prec):
    """Without bin buffers the last GEMM selects the top-C candidates itself
    (nothing stored); the records must equal those of the stored-bin path
    exactly, ties (integer entries) included."""
    m = cq()
    rng = np.random.default_rng(5)
    insts = []
    cm, E = syn.chain_instance(81, [2, 1], [6, 7, 5])
    insts.append(instance(cm, E, dd.initial_states(cm, [3, 2, 2]), [3, 2, 2]))
    cm = syn.chain_cutmap([1, 2], [5, 5, 6])
    E = [syn.integer_entries(rng, k, n, lo=-2, hi=3) for k, n in zip(syn.chain_ks([1, 2], 3), [5, 5, 6])]
    insts.append(instance(cm, E, dd.initial_states(cm, [2, 2, 2]), [2, 2, 2]))
    cm, E = syn.chain_instance(82, [0, 2, 1], [4, 5, 4, 5])
    insts.append(instance(cm, E, dd.initial_states(cm, [2, 1, 2, 1]), [2, 1, 2, 1]))
    R = 5
    dt = torch.float64 if prec == "fp64" else torch.float32
    bins = []
    for inst in insts:
        A = max_bins_log2(inst["subs"], dd.initial_states(inst["subs"], inst["max_active"]),
                          inst["max_active"])
        bins += [torch.empty(2 ** A, dtype=dt, device=DEV) for _ in range(R)]
    stored, done_s = m.cq_reconstruct_dd(insts, prec, R, bins=bins)
    fused, done_f = m.cq_reconstruct_dd(insts, prec, R)
    assert done_s == done_f
    assert strip_tiles(stored) == strip_tiles(fused)
    check_tile_counts(fused, stored)


def test_parallel_lanes_graph_and_direct_agree_with_single_instances():
    """Without bin buffers the instances of a batch run on parallel lanes
    (graph branches): both launch modes must reproduce, record for record,
    each instance run on its own."""
    m = cq()
    insts = []
    for i, (bonds, ns) in enumerate([([2, 1], [5, 6, 4]), ([1, 1, 1], [4, 3, 4, 3]), ([0, 2], [4, 5, 5]),
                                     ([1, 2], [5, 4, 5]), ([2, 2], [4, 5, 4]), ([1, 0, 1], [3, 4, 4, 3])]):
        cm, E = syn.chain_instance(120 + i, bonds, ns)
        M = [2] * len(ns)
        insts.append(instance(cm, E, dd.initial_states(cm, M), M))
    R = 4
    alone = [m.cq_reconstruct_dd([x], "fp32", R) for x in insts]
    for launch in ("graph", "direct"):
        recs, done = m.cq_reconstruct_dd(insts, "fp32", R, launch=launch)
        assert done == [d[1][0] for d in alone]
        assert recs == [d[0][0] for d in alone]


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
@pytest.mark.parametrize("case", ["int_2^21", "int_2^18x4", "dirichlet_2^21"])
def test_fused_top_c_matches_stored_bins_many_tiles(case, prec):
    """The fused top-C path across many tiles of the last GEMM: 2^18 to 2^21
    bins per recursion (16 to 128 output tiles of 128 x 128), so the tile
    bounds, the warm-up that raises the threshold and the pruned tile list
    all act across tiles.  Integer entries (few distinct values, many ties
    across tiles) make every bin exact, so the records must equal the stored
    path's and the oracle's bit for bit; on Dirichlet entries fused and stored
    must still agree exactly."""
    m = cq()
    rng = np.random.default_rng(6)
    if case == "int_2^21":      # recursion 0 has 2^21 bins, three merged outputs each
        bonds, ns, M, lo, hi = [1, 1], [10, 10, 10], [7, 7, 7], -2, 3
    elif case == "int_2^18x4":  # four recursions of 2^18 bins, ties everywhere
        bonds, ns, M, lo, hi = [1, 1], [12, 12, 12], [6, 6, 6], -1, 1
    else:
        bonds, ns, M, lo, hi = [2, 2], [10, 10, 10], [7, 7, 7], None, None
    if lo is None:
        cm, E = syn.chain_instance(83, bonds, ns)
    else:
        cm = syn.chain_cutmap(bonds, ns)
        E = [syn.integer_entries(rng, k, n, lo=lo, hi=hi) for k, n in zip(syn.chain_ks(bonds, 3), ns)]
    R = 4
    st = dd.initial_states(cm, M)
    inst = instance(cm, E, st, M)
    dt = torch.float64 if prec == "fp64" else torch.float32
    A = max_bins_log2(cm, st, M)
    bins = [torch.full((2 ** A,), float("nan"), dtype=dt, device=DEV) for _ in range(R)]
    print(f"fused vs stored {case} {prec}: 2^{A} bins", flush=True)
    stored, done_s = m.cq_reconstruct_dd([inst], prec, R, bins=bins)
    fused, done_f = m.cq_reconstruct_dd([inst], prec, R)
    torch.cuda.synchronize()
    assert done_s == done_f == [R]
    assert strip_tiles(stored) == strip_tiles(fused)
    check_tile_counts(fused, stored)
    run = sum(r["tiles_run"] for r in fused[0])
    print(f"  tiles run {run} of {sum(r['tiles'] for r in fused[0])}", flush=True)
    if lo is not None:
        compare(cm, E, st, M, R, prec, tol=0)


# --- breadth-first query -------------------------------------------------------

def _bfs_compare(cm, E, M, levels, width, prec, tol, exact):
    """GPU nodes against the oracle's: level, parent, parent bin, labels,
    FP64 total and candidates (bins exact; values exact or within tol)."""
    st0 = dd.initial_states(cm, M)
    ref = dd.run_bfs(cm, E, st0, M, levels, width)
    print(f"bfs {prec} levels {levels} width {width}: {len(ref)} nodes", flush=True)
    got = cq().cq_reconstruct_dd_bfs(instance(cm, E, st0, M), prec, levels, width)
    torch.cuda.synchronize()
    assert len(got) == len(ref)
    for g, r in zip(got, ref):
        assert (g["level"], g["parent"], g["parent_bin"]) == (r["level"], r["parent"], r["parent_bin"])
        assert g["active"] == [mask(s.active) for s in r["states"]]
        assert g["merged"] == [mask(s.merged) for s in r["states"]]
        assert g["fixed"] == [mask(s.fixed.keys()) for s in r["states"]]
        assert g["fixed_vals"] == [mask(p for p, v in s.fixed.items() if v) for s in r["states"]]
        assert [b for (_, _, b) in g["list"]] == [i for (_, i) in r["candidates"]]
        vals = [v for (v, _, _) in g["list"]]
        want = [v for (v, _) in r["candidates"]]
        if exact:
            assert g["total"] == r["total"] and vals == want
        else:
            assert abs(g["total"] - r["total"]) <= tol
            assert np.max(np.abs(np.array(vals) - np.array(want)), initial=0.0) <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(3))
def test_bfs_integer_entries_exact(case, prec):
    rng = np.random.default_rng(70 + case)
    bonds = [int(rng.integers(1, 3)), int(rng.integers(1, 3))]
    ns = [5, 4, 5]
    cm = syn.chain_cutmap(bonds, ns)
    E = [syn.integer_entries(rng, k, n, lo=0, hi=3) for k, n in zip(syn.chain_ks(bonds, 3), ns)]
    _bfs_compare(cm, E, [1, 2, 1], levels=3, width=4, prec=prec, tol=0.0, exact=True)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-7)])
def test_bfs_dirichlet_chain(prec, tol):
    cm, E = syn.chain_instance(17, [2, 2], [5, 5, 5])
    _bfs_compare(cm, E, [2, 1, 2], levels=4, width=5, prec=prec, tol=tol, exact=False)


def test_bfs_arguments_rejected_before_launch():
    m = cq()
    cm, E = syn.chain_instance(3, [1], [3, 3])
    inst = instance(cm, E, dd.initial_states(cm, [1, 1]), [1, 1])
    for kw in (dict(levels=0, width=2), dict(levels=2, width=0), dict(levels=2, width=17)):
        with pytest.raises(m.CQError):
            m.cq_reconstruct_dd_bfs(inst, "fp64", **kw)


# --- the hand-worked case of Algorithm 1 ---------------------------------------

def _golden():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "dd_algorithm1.json")) as f:
        g = json.load(f)
    inst = g["instance"]
    subs = [(s["width"], list(s["init_cut"]), list(s["meas_cut"])) for s in inst["subcircuits"]]
    dev_inst = dict(subs=subs, entries=[to_dev(np.array(e, dtype=np.float64)) for e in inst["entries"]],
                    active=inst["active"], merged=inst["merged"], fixed=inst["fixed"],
                    fixed_vals=inst["fixed_vals"], max_active=inst["max_active"])
    return g, dev_inst


@pytest.mark.parametrize("launch", ["graph", "direct"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "bf16_split", "fp16", "fp16_split"])
def test_hand_worked_algorithm1(prec, launch):
    """The device run reproduces the case worked by hand from Algorithm 1:
    masks, bins, totals, L after every update (with the tie across
    recursions resolved by the truncation) and the pops.  The entries are
    small integers, exact in every precision."""
    g, inst = _golden()
    R = g["algorithm1"]["R"]
    want = g["algorithm1"]["recursions"]
    dt = torch.float64 if prec == "fp64" else torch.float32
    bins = [torch.full((16,), float("nan"), dtype=dt, device=DEV) for _ in range(R)]
    recs, done = cq().cq_reconstruct_dd([inst], prec, R, bins=bins, launch=launch)
    torch.cuda.synchronize()
    assert done == [len(want)]
    for r, (w, rec) in enumerate(zip(want, recs[0])):
        assert (rec["active"], rec["merged"], rec["fixed"], rec["fixed_vals"]) == \
            (w["active"], w["merged"], w["fixed"], w["fixed_vals"]), r
        assert rec["n_active"] == 2
        assert bins[r][:4].cpu().double().tolist() == [float(x) for x in w["bins"]], r
        assert rec["total"] == w["total"], r
        assert [[v, rr, b] for (v, rr, b) in rec["list"]] == w["L"], r
        assert rec["popped"]
    # without bin buffers the fused top-C path must keep the same records
    fused, done_f = cq().cq_reconstruct_dd([inst], prec, R, launch=launch)
    assert done_f == done and strip_tiles(fused) == strip_tiles(recs)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16_split"])
def test_hand_worked_bfs(prec):
    g, inst = _golden()
    want = g["bfs"]["nodes"]
    got = cq().cq_reconstruct_dd_bfs(inst, prec, g["bfs"]["levels"], g["bfs"]["width"])
    torch.cuda.synchronize()
    assert len(got) == len(want)
    for k, (w, nd) in enumerate(zip(want, got)):
        assert (nd["level"], nd["parent"], nd["parent_bin"]) == (w["level"], w["parent"], w["parent_bin"]), k
        assert (nd["active"], nd["merged"], nd["fixed"], nd["fixed_vals"]) == \
            (w["active"], w["merged"], w["fixed"], w["fixed_vals"]), k
        assert nd["total"] == w["total"], k
        assert [[v, b] for (v, _, b) in nd["list"]] == w["candidates"], k


def test_graph_cache_reuse_and_eviction():
    """A batch repeated with the same launch parameters reuses its
    instantiated graph (same records); batches with other parameters fill the
    cache past its capacity, evicting graphs captured across parallel lanes;
    the first batch then runs again (captured anew) with the same records."""
    m = cq()
    ws_keep = []

    def batch(seed):
        insts = []
        for i, (bonds, ns) in enumerate([([2, 1], [5, 6, 4]), ([1, 1, 1], [4, 3, 4, 3]), ([0, 2], [4, 5, 5])]):
            cm, E = syn.chain_instance(seed + i, bonds, ns)
            M = [2] * len(ns)
            insts.append(instance(cm, E, dd.initial_states(cm, M), M))
        return insts

    first = batch(300)
    ws = torch.empty(m.cq_dd_workspace_size(first, "fp32", 4), dtype=torch.uint8, device=DEV)
    ref = m.cq_reconstruct_dd(first, "fp32", 4, workspace=ws)
    again = m.cq_reconstruct_dd(first, "fp32", 4, workspace=ws)
    assert again == ref
    for k in range(12):  # more distinct multi-lane batches than the cache keeps
        other = batch(310 + 3 * k)
        w = torch.empty(m.cq_dd_workspace_size(other, "fp32", 3), dtype=torch.uint8, device=DEV)
        ws_keep.append(w)
        m.cq_reconstruct_dd(other, "fp32", 3, workspace=w)
    torch.cuda.synchronize()
    assert m.cq_reconstruct_dd(first, "fp32", 4, workspace=ws) == ref


# --- checkpoint and resume -----------------------------------------------------

@pytest.mark.parametrize("launch", ["graph", "direct"])
@pytest.mark.parametrize("split", [1, 3])
def test_checkpoint_and_resume_continue_algorithm1(launch, split):
    """Algorithm 1's state between recursions is the list L and the next
    recursion index (with the masks it zooms into).  A run split over two
    calls -- the first stopping after `split` recursions and saving that
    state, the second resuming from it -- takes the very recursions one call
    takes: the records agree field by field, recursion indices continue, and
    a third call from the final state runs nothing.  Integer entries (exact,
    with ties), a batch of two instances advancing in lockstep."""
    m = cq()
    rng = np.random.default_rng(71)
    insts = []
    for bonds, ns, M in (([1, 1], [4, 5, 4], [2, 1, 2]), ([2, 1], [4, 4, 5], [1, 2, 1])):
        cm = syn.chain_cutmap(bonds, ns)
        E = [syn.integer_entries(rng, k, n, lo=-3, hi=6) for k, n in zip(syn.chain_ks(bonds, 3), ns)]
        insts.append(instance(cm, E, dd.initial_states(cm, M), M))
    R = 5
    print(f"resume {launch} split {split}", flush=True)
    full, done_full = m.cq_reconstruct_dd(insts, "fp64", R, launch=launch)
    a, done_a, ck = m.cq_reconstruct_dd(insts, "fp64", R, launch=launch, recursions=split, checkpoint=True)
    assert len(ck) == 2 * m.cq_dd_checkpoint_bytes()
    b, done_b, ck2 = m.cq_reconstruct_dd(insts, "fp64", R, launch=launch, resume=ck, checkpoint=True)
    for i in range(2):
        assert done_a[i] == min(split, done_full[i])
        assert done_a[i] + done_b[i] == done_full[i]
        assert a[i] + b[i] == full[i]
        assert [r["recursion"] for r in a[i] + b[i]] == list(range(done_full[i]))
    c, done_c = m.cq_reconstruct_dd(insts, "fp64", R, launch=launch, resume=ck2)
    assert done_c == [0, 0] and c == [[], []]
    # the stored-bin path resumes the same way
    A = max(max_bins_log2(x["subs"], dd.initial_states(x["subs"], x["max_active"]), x["max_active"])
            for x in insts)
    bins = [torch.empty(2 ** A, dtype=torch.float64, device=DEV) for _ in range(2 * R)]
    sa, sdone_a, sck = m.cq_reconstruct_dd(insts, "fp64", R, bins=bins, launch=launch, recursions=split,
                                           checkpoint=True)
    sb, sdone_b = m.cq_reconstruct_dd(insts, "fp64", R, bins=bins, launch=launch, resume=sck)
    for i in range(2):
        assert strip_tiles([sa[i] + sb[i]]) == strip_tiles([full[i]])
