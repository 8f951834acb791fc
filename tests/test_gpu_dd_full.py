"""Batched dynamic definition at full size: 16 chain instances of four
20-output subcircuits (80 output qubits), K uniform in 2..6 with at most four
cuts per subcircuit, 8 active qubits per subcircuit (2^32 bins per recursion)
and R = 4 recursions, all captured in one graph.

The oracle cannot build 2^32 bins, so the checks are the ones it can do at
any size:

* every list value (FP64) against the oracle's value of that bin, from the
  entry columns the bin needs, merged and contracted by the oracle;
* the zoom chain: recursion r's masks follow from the bin popped at r - 1
  by the oracle's child/zoom rules;
* a recursion's FP64 total equals the value of the bin it zoomed into (its
  bins partition that bin), and recursion 0's total equals the closed form
  2^-K sum_l prod_c rowsum_c(l) for the smallest instance;
* with stored bins, a grid of 16^4 bins per recursion against the oracle,
  and the recursion's candidates and appended bins against the stored bins:
  the candidates are the C largest stored bins (value, then index), the
  appended bins the R largest of those by the oracle's value, and the gap
  between the R-th and the C-th stored value exceeds the error bound, so no
  bin outside the stored top C can belong to the true top R.
"""
import numpy as np
import pytest

from oracle import dd
from oracle.reconstruct import fd_contract
from workloads import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SEED = 400          # instance i uses seed SEED + i; the bond splits use SEED
N_INST = 16
N_OUT = 20
M_ACT = 8
R = 4


def fp32_floor(n_sub, K):
    """Absolute error an FP32 contraction can add below FP32's normal range,
    for operands of magnitude at most 1 (every entry here, merged or not, is
    bounded by its identity row, a Dirichlet draw).  Each elementary step
    (the conversion of an operand, a product, an addition) that flushes or
    rounds a result below 2^-126 adds at most 2^-126; the output is a sum of
    4^K label terms of n_sub factors each, and an error injected at a step
    reaches the output multiplied by at most the number of label terms that
    use it (every other factor is at most 1 in magnitude, 2^-K at most 1), so
    the sum over the at most (3 n_sub + 1) steps per term bounds it."""
    return (3 * n_sub + 1) * 4.0 ** K * 2.0 ** -126


def cq():
    import paper_2205_05836_amd as m
    return m


def batch():
    return syn.dd_batch_bonds(SEED, n_inst=N_INST, n_sub=4, k_range=(2, 6), max_k_per_sub=4)


def make_instance(i, bonds):
    ks = syn.chain_ks(bonds, 4)
    cm = syn.chain_cutmap(list(bonds), [N_OUT] * 4)
    ents = [syn.entries_torch(SEED + i, c, ks[c], N_OUT, DEV) for c in range(4)]
    M = [M_ACT] * 4
    st = dd.initial_states(cm, M)
    mask = lambda ps: sum(1 << p for p in ps)
    inst = dict(subs=cm, entries=ents, active=[mask(s.active) for s in st],
                merged=[mask(s.merged) for s in st], fixed=[0] * 4, fixed_vals=[0] * 4,
                max_active=M)
    return inst, cm, ks


def states_of(rec):
    """Oracle SubStates from a record's masks."""
    out = []
    for a, m, f, fv in zip(rec["active"], rec["merged"], rec["fixed"], rec["fixed_vals"]):
        bits = lambda x: [p for p in range(N_OUT) if (x >> p) & 1]
        out.append(dd.SubState(bits(a), bits(m), {p: (fv >> p) & 1 for p in bits(f)}))
    return out


def local_problem(seed, bonds, ks, states, samples):
    """Entries restricted to sampled active values.  Subcircuit c gets 16
    sample slots (4 local bits, the first local outputs) followed by its
    merged outputs; column (s, m) holds the full entry column whose active
    bits are samples[c][s], fixed bits their values and merged bits m.  The
    oracle then merges and contracts these local tensors; local bin
    (s_0, s_1, s_2, s_3) is the full bin made of the sampled values."""
    locs, lstates, n_locs = [], [], []
    for c, st in enumerate(states):
        act, mer = sorted(st.active), sorted(st.merged)
        na, nm = len(act), len(mer)
        S = list(samples[c]) + [samples[c][0]] * (16 - len(samples[c]))
        cols = np.zeros((16, 1 << nm), dtype=np.int64)
        base = 0
        for p, v in st.fixed.items():
            base |= v << (N_OUT - 1 - p)
        m = np.arange(1 << nm, dtype=np.int64)
        mbits = np.zeros(1 << nm, dtype=np.int64)
        for i, p in enumerate(mer):
            mbits |= ((m >> (nm - 1 - i)) & 1) << (N_OUT - 1 - p)
        for s, a in enumerate(S):
            abits = 0
            for i, p in enumerate(act):
                abits |= ((a >> (na - 1 - i)) & 1) << (N_OUT - 1 - p)
            cols[s] = base | abits | mbits
        flat = cols.ravel()
        uniq, inv = np.unique(flat, return_inverse=True)
        E = syn.entries_columns(seed, c, ks[c], N_OUT, uniq)[:, inv]
        locs.append(E)
        lstates.append(dd.SubState(list(range(4)), list(range(4, 4 + nm)), {}))
        n_locs.append(4 + nm)
    cm_loc = syn.chain_cutmap(list(bonds), n_locs)
    reduced = [dd.merge_entries(E, n, st) for E, n, st in zip(locs, n_locs, lstates)]
    return cm_loc, reduced


def grid_values(cm_loc, reduced, absolute=False):
    ops = [np.abs(r) for r in reduced] if absolute else reduced
    return fd_contract(cm_loc, ops)  # 16^4 local bins, subcircuit 0 most significant


def split_bin(b, states):
    parts, shift = [], sum(len(st.active) for st in states)
    for st in states:
        shift -= len(st.active)
        parts.append((b >> shift) & ((1 << len(st.active)) - 1))
    return parts


@pytest.fixture(scope="module")
def full_batch():
    bonds_all = batch()
    insts, meta = [], []
    for i, bonds in enumerate(bonds_all):
        inst, cm, ks = make_instance(i, bonds)
        insts.append(inst)
        meta.append((bonds, ks, cm))
    torch.cuda.synchronize()
    print(f"dd batch of {N_INST} instances built", flush=True)
    return insts, meta


@pytest.mark.parametrize("prec", ["fp32", "bf16_split", "fp16_split", "fp64"])
def test_batch_full_size_lists_zoom_and_totals(prec, full_batch):
    m = cq()
    insts, meta = full_batch
    recs, done = m.cq_reconstruct_dd(insts, prec, R)
    print(f"dd batch {prec} done: {done}", flush=True)
    # with 20 outputs and 8 activated per zoom, L never runs empty before R
    assert done == [R] * N_INST
    M = [M_ACT] * 4
    for i, (bonds, ks, cm) in enumerate(meta):
        rr = recs[i]
        assert len(rr) == R
        # zoom chain and totals
        st0 = dd.initial_states(cm, M)
        assert [s.active for s in states_of(rr[0])] == [s.active for s in st0]
        for r in range(1, len(rr)):
            v, rec, b = rr[r - 1]["list"][0]
            assert rr[r - 1]["popped"]
            want = dd.zoom(dd.child_states(states_of(rr[rec]), b), M)
            got = states_of(rr[r])
            assert [(s.active, s.merged, s.fixed) for s in got] == \
                   [(s.active, s.merged, s.fixed) for s in want], (i, r)
            assert abs(rr[r]["total"] - v) <= 1e-12 * max(abs(v), 1e-300) + 1e-300, (i, r)
        # every listed bin against the oracle, grouped by its recursion
        by_rec = {}
        for r in range(len(rr)):
            for (v, rec, b) in rr[r]["list"]:
                by_rec.setdefault(rec, {})[b] = v
        for rec, vals in by_rec.items():
            states = states_of(rr[rec])
            bins = sorted(vals)
            parts = [split_bin(b, states) for b in bins]
            samples = [sorted(set(p[c] for p in parts)) for c in range(4)]
            cm_loc, red = local_problem(SEED + i, bonds, ks, states, samples)
            grid = grid_values(cm_loc, red).reshape(16, 16, 16, 16)
            for b, p in zip(bins, parts):
                ref = grid[tuple(samples[c].index(p[c]) for c in range(4))]
                assert abs(vals[b] - ref) <= 1e-10, (i, rec, b, vals[b], ref)
    # recursion-0 total of the smallest instance: closed form over full row sums
    i = int(np.argmin([sum(4 ** k for k in ks) for (_, ks, _) in meta]))
    bonds, ks, cm = meta[i]
    rs = [syn.dirichlet_entries(SEED + i, c, ks[c], N_OUT).sum(axis=1) for c in range(4)]
    tot = float(fd_contract(cm, [r[:, None] for r in rs])[0])
    assert abs(recs[i][0]["total"] - tot) <= 1e-12 * abs(tot) + 1e-15, (recs[i][0]["total"], tot)


def stored_top(b, k, chunk=1 << 28):
    """The k largest stored bins, value descending then index ascending
    (torch.topk per chunk, then an exact host sort of the survivors)."""
    vals, idxs = [], []
    for off in range(0, b.numel(), chunk):
        part = b[off: off + chunk]
        kk = min(k + 8, part.numel())
        v, i = torch.topk(part, kk)
        vals.append(v.double().cpu().numpy())
        idxs.append(i.cpu().numpy().astype(np.int64) + off)
    v, i = np.concatenate(vals), np.concatenate(idxs)
    order = sorted(range(len(v)), key=lambda j: (-v[j], i[j]))[:k]
    return v[order], i[order]


def check_top_r_against_stored(b, rec, r, Rcap, states, bonds, ks, seed, rel, floor):
    """Recursion r (every bin still has merged outputs) keeps the C = 4R
    largest bins in working precision as candidates, re-evaluates them in
    FP64 and appends the R largest; the entries of L that came from r are a
    prefix of those.  The candidates are checked exactly against the stored
    bins, the appended ones against the oracle's values of the candidates,
    and the gap between the R-th and the C-th stored value against the
    rounding bound, which shows that the true R largest of all bins are among
    the candidates."""
    C = min(4 * Rcap, 64)
    sv, si = stored_top(b, C)
    parts = [split_bin(int(x), states) for x in si]
    samples = [sorted(set(p[c] for p in parts)) for c in range(4)]
    assert all(len(x) <= 16 for x in samples)
    cm_loc, red = local_problem(seed, bonds, ks, states, samples)
    ref = grid_values(cm_loc, red).reshape(16, 16, 16, 16)
    scl = grid_values(cm_loc, red, absolute=True).reshape(16, 16, 16, 16)
    pos = [tuple(samples[c].index(p[c]) for c in range(4)) for p in parts]
    true = np.array([ref[q] for q in pos])
    bound = np.array([rel * scl[q] + floor for q in pos])
    # the stored candidates are correct to the rounding bound
    assert np.all(np.abs(sv - true) <= bound), (r, np.max(np.abs(sv - true) / bound))
    # the R largest candidates by the oracle's value (desc, then bin asc)
    best = sorted(range(C), key=lambda j: (-true[j], si[j]))[:Rcap]
    mine = [(v, b_) for (v, rr_, b_) in rec["list"] if rr_ == r]
    assert 1 <= len(mine) <= Rcap
    for j, (v, b_) in enumerate(mine):
        k = best[j]
        assert abs(v - true[k]) <= 1e-10, (r, j, v, true[k])
        gap_lo = j == 0 or abs(true[best[j - 1]] - true[k]) > 2e-10
        gap_hi = j + 1 >= len(best) or abs(true[best[j + 1]] - true[k]) > 2e-10
        if gap_lo and gap_hi:
            assert b_ == int(si[k]), (r, j, b_, int(si[k]))
    # no bin outside the candidates can reach the R-th largest true value
    margin = sv[Rcap - 1] - sv[C - 1]
    print(f"recursion {r}: stored top {C} from {sv[0]:.4e} to {sv[C - 1]:.4e}; "
          f"R-th minus C-th {margin:.3e} against a bound of {2 * bound.max():.3e}", flush=True)
    assert margin > 2 * bound.max()


@pytest.mark.parametrize("prec", ["fp32", "fp16_split", "fp64"])
def test_largest_instance_stored_bins_grid(prec):
    """Stored bins of the batch's largest instance on a 16^4 grid of sampled
    active values against the oracle.  FP16-split runs with the per-label
    balance and the column scaling of the reduced entries; its bound relative
    to each bin's |E| scale is the same 1e-5 as FP32's: hi + lo keeps 22 bits
    of every scaled operand, and an operand flushed below FP16's range costs
    at most 2^-25 of its column's largest value, whose term (the identity
    row bounds every row of these entries) is part of the bin's scale."""
    m = cq()
    bonds_all = batch()
    i = int(np.argmax([sum(4 ** k for k in syn.chain_ks(b, 4)) for b in bonds_all]))
    bonds = bonds_all[i]
    inst, cm, ks = make_instance(i, bonds)
    R2 = 2
    dt = torch.float64 if prec == "fp64" else torch.float32
    bins = [torch.empty(2 ** (4 * M_ACT), dtype=dt, device=DEV) for _ in range(R2)]
    print(f"dd instance {i} bonds {bonds} stored bins {prec}", flush=True)
    recs, done = m.cq_reconstruct_dd([inst], prec, R2, bins=bins)
    rr = recs[0]
    assert done[0] == R2
    rng = np.random.default_rng(77)
    for r in range(R2):
        states = states_of(rr[r])
        na = [len(s.active) for s in states]
        assert rr[r]["n_active"] == sum(na) == 4 * M_ACT
        # 16 sampled active values per subcircuit: extremes, the listed bins' values, random
        listed = [split_bin(b, states) for (_, rec, b) in rr[r]["list"] if rec == r]
        samples = []
        for c in range(4):
            s = {0, (1 << na[c]) - 1} | {p[c] for p in listed}
            while len(s) < 16:
                s.add(int(rng.integers(0, 1 << na[c])))
            samples.append(sorted(s)[:16])
        cm_loc, red = local_problem(SEED + i, bonds, ks, states, samples)
        ref = grid_values(cm_loc, red)
        scale = grid_values(cm_loc, red, absolute=True)
        idx = np.zeros(16 ** 4, dtype=np.int64)
        for g in range(16 ** 4):
            s = [(g >> (4 * (3 - c))) & 15 for c in range(4)]
            v = 0
            for c in range(4):
                v = (v << na[c]) | samples[c][s[c]]
            idx[g] = v
        got = bins[r][torch.from_numpy(idx).to(DEV)].cpu().numpy().astype(np.float64)
        err = np.abs(got - ref)
        print(f"recursion {r}: max abs err {err.max():.3e}, max |bin| {np.abs(ref).max():.3e}, "
              f"max err/scale {np.max(err / np.maximum(scale, 1e-300)):.3e}", flush=True)
        K = sum(bonds)
        floor = 1e-300 if prec == "fp64" else fp32_floor(4, K)
        rel = 1e-13 if prec == "fp64" else 1e-5
        if prec == "fp64":
            assert err.max() < 1e-10
        else:
            assert err.max() < 1e-6
        assert np.all(err <= rel * scale + floor)
        check_top_r_against_stored(bins[r][: 2 ** sum(na)], rr[r], r, R2, states, bonds, ks,
                                   SEED + i, rel, floor)
        # the recursion total against the sum of the bins (FP64 from the GPU's own bins)
        s = float(torch.sum(bins[r][: 2 ** sum(na)], dtype=torch.float64).item())
        assert abs(s - rr[r]["total"]) <= (1e-9 if prec == "fp64" else 1e-5)


def test_bfs_full_size_candidates_and_children():
    """Breadth-first query at full size on instance 0 of the batch (four
    20-output subcircuits, 8 active outputs each: 2^32 bins per node), three
    levels of width 3.  Every node's candidate values against the oracle
    (local problem of the sampled bins), every child's FP64 total against
    the candidate value of the parent bin it refines, and the level
    structure (level 1 zooms into the root's candidates in order)."""
    m = cq()
    bonds = batch()[0]
    inst, cm, ks = make_instance(0, bonds)
    W = 3
    print(f"bfs full size, bonds {bonds}", flush=True)
    nodes = m.cq_reconstruct_dd_bfs(inst, "fp32", levels=3, width=W)
    torch.cuda.synchronize()
    assert nodes[0]["level"] == 0 and nodes[0]["parent"] == -1
    lv1 = [nd for nd in nodes if nd["level"] == 1]
    assert [nd["parent_bin"] for nd in lv1] == [b for (_, _, b) in nodes[0]["list"][:W]]
    for k, nd in enumerate(nodes):
        if nd["parent"] >= 0:
            par = nodes[nd["parent"]]
            v = {b: val for (val, _, b) in par["list"]}[nd["parent_bin"]]
            assert abs(nd["total"] - v) <= 1e-12 * max(abs(v), 1e-300) + 1e-300, (k, nd["total"], v)
        if not nd["list"]:
            continue
        states = states_of(nd)
        bins = [b for (_, _, b) in nd["list"]]
        parts = [split_bin(b, states) for b in bins]
        samples = [sorted(set(p[c] for p in parts)) for c in range(4)]
        cm_loc, red = local_problem(SEED, bonds, ks, states, samples)
        grid = grid_values(cm_loc, red).reshape(16, 16, 16, 16)
        for (val, _, b), p in zip(nd["list"], parts):
            ref = grid[tuple(samples[c].index(p[c]) for c in range(4))]
            assert abs(val - ref) <= 1e-10, (k, b, val, ref)
