"""Pins of the oracle's list handling in dynamic definition against a case
worked by hand from Algorithm 1 and the breadth-first query (Section 4.3):
tests/golden/dd_algorithm1.json gives, per recursion, the masks, every bin,
the bins appended to L, L after sorting and truncation to R, and the popped
entry; per breadth-first node, its masks, bins and candidates.  The case has
a tie across recursions that the truncation resolves and a tie inside one
node, so a slip in the append count, the sort keys, the truncation or the
zoom rule changes some recorded value."""
import json
import os

import numpy as np
import pytest

from oracle import cutmap
from oracle import dd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dd_algorithm1.json")


def load():
    with open(GOLDEN) as f:
        g = json.load(f)
    inst = g["instance"]
    subs = [(s["width"], list(s["init_cut"]), list(s["meas_cut"])) for s in inst["subcircuits"]]
    E = [np.array(e, dtype=np.float64) for e in inst["entries"]]
    return g, inst, subs, E


def states_of(subs, active, merged, fixed, fixed_vals):
    out = []
    for s, a, m, f, v in zip(subs, active, merged, fixed, fixed_vals):
        n = len(cutmap.outputs(s))
        out.append(dd.SubState([i for i in range(n) if (a >> i) & 1],
                               [i for i in range(n) if (m >> i) & 1],
                               {i: (v >> i) & 1 for i in range(n) if (f >> i) & 1}))
    return out


def masks_of(states):
    act = [sum(1 << i for i in st.active) for st in states]
    mer = [sum(1 << i for i in st.merged) for st in states]
    fix = [sum(1 << i for i in st.fixed) for st in states]
    val = [sum(v << i for i, v in st.fixed.items()) for st in states]
    return act, mer, fix, val


def test_golden_bins_add_up():
    """The hand-worked bins agree with themselves: every recursion's bins add
    to its total, and a child's total is the value of the bin it zooms into."""
    g, _, _, _ = load()
    recs = g["algorithm1"]["recursions"]
    for r in recs:
        assert sum(r["bins"]) == r["total"]
    for prev, nxt in zip(recs, recs[1:]):
        assert prev["popped"][0] == nxt["total"]
    for node in g["bfs"]["nodes"]:
        assert sum(node["bins"]) == node["total"]
        if node["parent"] >= 0:
            parent = g["bfs"]["nodes"][node["parent"]]
            assert parent["bins"][node["parent_bin"]] == node["total"]


def test_algorithm1_matches_hand_worked_records():
    g, inst, subs, E = load()
    st0 = states_of(subs, inst["active"], inst["merged"], inst["fixed"], inst["fixed_vals"])
    want = g["algorithm1"]["recursions"]
    got = dd.run(subs, E, st0, inst["max_active"], g["algorithm1"]["R"])
    assert len(got) == len(want)
    for r, (w, rec) in enumerate(zip(want, got)):
        assert masks_of(rec["states"]) == (w["active"], w["merged"], w["fixed"], w["fixed_vals"]), r
        assert np.array_equal(rec["bins"], np.array(w["bins"], dtype=np.float64)), r
        assert [list(e) for e in rec["L"]] == w["L"], r
        assert list(rec["popped"]) == w["popped"], r


def test_algorithm1_appends_the_r_largest_bins_with_merged_outputs():
    """The appended entries are the R largest bins (value desc, bin asc) of
    a recursion with merged outputs, none of one without."""
    g, inst, subs, E = load()
    R = g["algorithm1"]["R"]
    for r, w in enumerate(g["algorithm1"]["recursions"]):
        states = states_of(subs, w["active"], w["merged"], w["fixed"], w["fixed_vals"])
        bins = dd.bins_of(subs, E, states)
        if any(st.merged for st in states):
            order = sorted(range(len(bins)), key=lambda i: (-bins[i], i))[:R]
            assert [[float(bins[i]), r, i] for i in order] == w["appended"]
        else:
            assert w["appended"] == []


def test_bfs_matches_hand_worked_nodes():
    g, inst, subs, E = load()
    st0 = states_of(subs, inst["active"], inst["merged"], inst["fixed"], inst["fixed_vals"])
    want = g["bfs"]["nodes"]
    got = dd.run_bfs(subs, E, st0, inst["max_active"], g["bfs"]["levels"], g["bfs"]["width"])
    assert len(got) == len(want)
    for k, (w, nd) in enumerate(zip(want, got)):
        assert (nd["level"], nd["parent"], nd["parent_bin"]) == (w["level"], w["parent"], w["parent_bin"]), k
        assert masks_of(nd["states"]) == (w["active"], w["merged"], w["fixed"], w["fixed_vals"]), k
        assert np.array_equal(nd["bins"], np.array(w["bins"], dtype=np.float64)), k
        assert nd["total"] == pytest.approx(w["total"], abs=0)
        assert [list(c) for c in nd["candidates"]] == w["candidates"], k
