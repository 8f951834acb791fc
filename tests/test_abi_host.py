"""Host-only tests of the C ABI: the library loads and exports every symbol
the headers declare, validation rejects bad arguments before any launch, and
the contraction planner's GEMM/permute steps, replayed in numpy, reproduce
Eq. 1 as computed by the oracle on random cut graphs."""
import ctypes as C
import glob
import json
import os
import re

import numpy as np
import pytest

from oracle import cutmap
from oracle import reconstruct as rc
from workloads import circuits as wc
from workloads import synthetic as syn
from paper_2205_05836_amd._lib import FD_NOALLOC_SCRATCH_BYTES

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def lib():
    from paper_2205_05836_amd import _lib
    return _lib.lib()


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(cq_[a-z_0-9]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = lib()
    names = declared_symbols()
    assert {"cq_attribute", "cq_reconstruct_fd", "cq_reconstruct_dd", "cq_plan_json"} <= names
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    L = lib()
    L.cq_status_string.restype = C.c_char_p
    for code, name in [(0, b"CQ_OK"), (-3, b"CQ_ERR_CUTMAP"), (-7, b"CQ_ERR_HIP")]:
        assert L.cq_status_string(code) == name


def test_validate_reports_k_and_n():
    import paper_2205_05836_amd as cq
    cc = wc.two_way_circuit_20q(1)
    assert cq.validate_cutmap(cc.subcircuits()) == (4, 20)
    assert cq.validate_cutmap(syn.chain_cutmap([4, 4], [10, 10, 10])) == (8, 30)


BAD_MAPS = [
    ("missing end", [(2, [-1, -1], [0, -1]), (1, [-1], [-1])], -3),
    ("measured twice", [(2, [-1, -1], [0, 0]), (1, [0], [-1])], -3),
    ("self loop", [(2, [0, -1], [-1, 0])], -3),
    ("id gap", [(1, [-1], [1]), (1, [1], [-1])], -3),
    ("too wide", [(40, [-1] * 40, [-1] * 40)], -2),
    ("bad id", [(1, [-1], [-5]), (1, [-5], [-1])], -3),
    ("too many local cuts", [(9, [-1] * 9, list(range(9))), (9, list(range(9)), [-1] * 9)], -2),
]


@pytest.mark.parametrize("name,subs,code", BAD_MAPS, ids=[b[0] for b in BAD_MAPS])
def test_bad_cut_maps_rejected(name, subs, code):
    import paper_2205_05836_amd as cq
    with pytest.raises(cq.CQError) as e:
        cq.validate_cutmap(subs)
    assert e.value.status == code


def test_bad_precision_and_perm_rejected():
    from paper_2205_05836_amd import _lib
    from paper_2205_05836_amd.api import _Subs
    L = lib()
    cm = syn.chain_cutmap([1], [2, 2])
    s = _Subs(cm)
    b = C.c_size_t()
    assert L.cq_fd_workspace_size(2, s.ptr(), 9, None, C.byref(b)) == -1
    perm = (C.c_int32 * 4)(0, 1, 1, 3)
    assert L.cq_fd_workspace_size(2, s.ptr(), 0, perm, C.byref(b)) == -1
    assert L.cq_fd_workspace_size(0, s.ptr(), 0, None, C.byref(b)) == -1
    del _lib


def test_fd_rejects_before_launch_without_gpu():
    # invalid arguments are reported before anything touches the device
    from paper_2205_05836_amd.api import _Subs
    L = lib()
    cm = syn.chain_cutmap([1], [2, 2])
    s = _Subs(cm)
    fake = (C.c_void_p * 2)(0x1000, 0x2000)
    # null output
    assert L.cq_reconstruct_fd(2, s.ptr(), fake, 0, None, None, None, 0, None) == -1
    # workspace missing for a plan that needs one
    cm3 = syn.chain_cutmap([2, 2], [4, 4, 4])
    s3 = _Subs(cm3)
    b = C.c_size_t()
    assert L.cq_fd_workspace_size(3, s3.ptr(), 1, None, C.byref(b)) == 0 and b.value > 0
    fake3 = (C.c_void_p * 3)(0x1000, 0x2000, 0x3000)
    assert L.cq_reconstruct_fd(3, s3.ptr(), fake3, 1, None, C.c_void_p(0x4000), None, 0, None) == -5


def test_noalloc_rejects_before_launch_without_gpu():
    """The no-allocation entry point reports a workspace beyond its fixed
    scratch, and a bad cut map, before anything touches a device."""
    from paper_2205_05836_amd.api import _Subs
    L = lib()
    cm = syn.chain_cutmap([4, 4], [10, 10, 10])
    s = _Subs(cm)
    b = C.c_size_t()
    assert L.cq_fd_workspace_size(3, s.ptr(), 1, None, C.byref(b)) == 0
    assert b.value > FD_NOALLOC_SCRATCH_BYTES
    fake = (C.c_void_p * 3)(0x1000, 0x2000, 0x3000)
    assert L.cq_reconstruct_fd_noalloc(3, s.ptr(), fake, 1, None, C.c_void_p(0x4000), None) == -5
    assert b"scratch" in L.cq_last_error()
    bad = _Subs([(2, [-1, -1], [0, -1]), (2, [-1, -1], [-1, -1])])
    assert L.cq_reconstruct_fd_noalloc(2, bad.ptr(), fake, 1, None, C.c_void_p(0x4000), None) == -3


def test_fault_injection_stops_before_launch(monkeypatch):
    from paper_2205_05836_amd.api import _Subs
    L = lib()
    cm = syn.chain_cutmap([1], [2, 2])
    s = _Subs(cm)
    fake = (C.c_void_p * 2)(0x1000, 0x2000)
    monkeypatch.setenv("CQ_FAULT_INJECT", "fd")
    assert L.cq_reconstruct_fd(2, s.ptr(), fake, 0, None, C.c_void_p(0x4000), None, 0, None) == -7
    L.cq_last_error.restype = C.c_char_p
    assert b"injected" in L.cq_last_error()


def test_dd_mask_validation():
    import paper_2205_05836_amd as cq
    cm = syn.chain_cutmap([1], [3, 3])
    fake = [_FakeTensor(0x1000), _FakeTensor(0x2000)]
    base = dict(subs=cm, entries=fake, active=[0b011, 0b001], merged=[0b100, 0b110],
                fixed=[0, 0], fixed_vals=[0, 0], max_active=[1, 1])
    cq.cq_dd_workspace_size([base], "fp64", 2)
    bad = dict(base, merged=[0b110, 0b110])   # overlaps active
    with pytest.raises(cq.CQError) as e:
        cq.cq_dd_workspace_size([bad], "fp64", 2)
    assert e.value.status == -4
    bad = dict(base, merged=[0b000, 0b110])   # misses an output
    with pytest.raises(cq.CQError) as e:
        cq.cq_dd_workspace_size([bad], "fp64", 2)
    assert e.value.status == -4
    bad = dict(base, fixed_vals=[0b100, 0])   # value on a non-fixed output
    with pytest.raises(cq.CQError) as e:
        cq.cq_dd_workspace_size([bad], "fp64", 2)
    assert e.value.status == -4
    with pytest.raises(cq.CQError) as e:
        cq.cq_dd_workspace_size([base], "fp64", 0)
    assert e.value.status == -1


def test_dd_resume_checkpoint_validated_before_launch():
    """A checkpoint that no run of the instance could have written -- masks
    that do not partition the outputs (all zero), or a recursion index out of
    range (all ones) -- is rejected with CQ_ERR_ARG before any launch."""
    import paper_2205_05836_amd as cq
    from paper_2205_05836_amd import _lib
    from paper_2205_05836_amd.api import _Instances
    cm = syn.chain_cutmap([1], [3, 3])
    fake = [_FakeTensor(0x1000), _FakeTensor(0x2000)]
    base = dict(subs=cm, entries=fake, active=[0b011, 0b001], merged=[0b100, 0b110],
                fixed=[0, 0], fixed_vals=[0, 0], max_active=[1, 1])
    ck = cq.cq_dd_checkpoint_bytes()
    assert ck > 0
    ins = _Instances([base])
    recs = (_lib.cq_dd_record * 2)()
    done = (C.c_int32 * 1)()
    ws = C.create_string_buffer(1 << 16)
    for fill in (b"\x00", b"\xff"):
        blob = C.create_string_buffer(fill * ck, ck)
        par = _lib.cq_dd_params(_lib.PRECISION["fp64"], 2, 0, 0, C.cast(blob, C.c_void_p), None)
        st = lib().cq_reconstruct_dd(1, ins.arr, C.byref(par), recs, None, done,
                                     C.cast(ws, C.c_void_p), C.c_size_t(1 << 16), None)
        assert st == -1, (fill, st)
        assert "resume checkpoint" in lib().cq_last_error().decode()
    par = _lib.cq_dd_params(_lib.PRECISION["fp64"], 2, 0, -1, None, None)
    st = lib().cq_reconstruct_dd(1, ins.arr, C.byref(par), recs, None, done, C.cast(ws, C.c_void_p),
                                 C.c_size_t(1 << 16), None)
    assert st == -1


class _FakeTensor:
    def __init__(self, p):
        self.p = p

    def data_ptr(self):
        return self.p


# ---------------------------------------------------------------------------
# Planner replay
# ---------------------------------------------------------------------------

def plan_json(subs, prec="fp64", out_bits=None, out_perm=None):
    from paper_2205_05836_amd.api import _Subs
    L = lib()
    s = _Subs(subs)
    ob = (C.c_int32 * len(subs))(*out_bits) if out_bits is not None else None
    op = (C.c_int32 * len(out_perm))(*out_perm) if out_perm is not None else None
    need = C.c_size_t()
    st = L.cq_plan_json(len(subs), s.ptr(), {"fp64": 0, "fp32": 1}[prec], ob, op, None, 0,
                        C.byref(need))
    assert st == -1 and need.value > 0
    buf = C.create_string_buffer(need.value)
    assert L.cq_plan_json(len(subs), s.ptr(), {"fp64": 0, "fp32": 1}[prec], ob, op, buf,
                          need.value, C.byref(need)) == 0
    return json.loads(buf.value.decode())


def replay(plan, inputs):
    """Executes the planned steps with numpy (float64)."""
    bufs = {}

    def buf(tid):
        t = plan["tensors"][tid]
        if t["loc"] == "input":
            a = inputs[t["index"]].ravel()
            assert a.size == t["elems"]
            return a
        key = "out" if t["loc"] == "out" else ("work", t["index"])
        if key not in bufs:
            bufs[key] = np.zeros(t["elems"])
        return bufs[key]

    for s in plan["steps"]:
        if s["op"] == "gemm":
            A, B, Cb = buf(s["a"]), buf(s["b"]), buf(s["c"])
            z = np.arange(s["Z"])[:, None, None]
            k = np.arange(s["K"])[None, :, None]
            ia = z * s["sAz"] + k * s["sAk"] + np.arange(s["M"])[None, None, :]
            ib = z * s["sBz"] + k * s["sBk"] + np.arange(s["N"])[None, None, :]
            prod = np.einsum("zkm,zkn->zmn", A[ia], B[ib]) * s["alpha"]
            ic = z * s["sCz"] + np.arange(s["M"])[None, :, None] * s["ldc"] + \
                np.arange(s["N"])[None, None, :]
            assert ia.max() < A.size and ib.max() < B.size and ic.max() < Cb.size
            Cb[ic] = prod
        else:
            src, dst = buf(s["src"]), buf(s["dst"])
            i = np.arange(dst.size, dtype=np.int64)
            off = np.zeros_like(i)
            r = i.copy()
            for l2, st in zip(reversed(s["log2"]), reversed(s["sstride"])):
                off += (r & ((1 << l2) - 1)) * st
                r >>= l2
            dst[:] = s["alpha"] * src[off]
    return bufs["out"]


def _random_graph_cases(count, seed0=3000):
    out, seed = [], seed0
    while len(out) < count:
        rng = np.random.default_rng(seed)
        seed += 1
        n_sub = int(rng.integers(2, 6))
        n = int(rng.integers(n_sub, 10))
        cc = wc.random_cut_circuit(rng, n, n_sub, int(rng.integers(1, 7)), depth=6)
        if cc is None or not cc.cuts:
            continue
        subs = cc.subcircuits()
        if max(len(cutmap.incident_cuts(s)) for s in subs) > 6:
            continue
        if sum(len(cutmap.outputs(s)) for s in subs) != n:
            continue
        out.append((seed, subs))
    return out


@pytest.mark.parametrize("seed,subs", _random_graph_cases(30))
def test_plan_replay_matches_oracle_on_random_cut_graphs(seed, subs):
    rng = np.random.default_rng(seed)
    E = [rng.standard_normal((4 ** len(cutmap.incident_cuts(s)), 2 ** len(cutmap.outputs(s))))
         for s in subs]
    ref = rc.fd_contract(subs, E)
    plan = plan_json(subs)
    got = replay(plan, E)
    assert np.max(np.abs(got - ref)) < 1e-10 * max(1.0, np.abs(ref).max())
    n = sum(len(cutmap.outputs(s)) for s in subs)
    perm = [int(x) for x in rng.permutation(n)]
    got = replay(plan_json(subs, out_perm=perm), E)
    assert np.max(np.abs(got - rc.apply_out_perm(ref, perm))) < 1e-10 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("bonds,ns,bits", [
    ([4, 4], [5, 5, 5], [2, 3, 1]),
    ([0, 3, 1], [3, 4, 4, 3], [0, 2, 4, 1]),
    ([2, 2, 2, 2], [2, 3, 2, 3, 2], [1, 1, 1, 1, 1]),
    ([3, 2, 3], [4, 4, 4, 4], [4, 4, 4, 4]),
])
def test_plan_replay_with_partial_outputs(bonds, ns, bits):
    # the dynamic-definition bin contraction plans over active-bit counts
    rng = np.random.default_rng(len(ns))
    cm = syn.chain_cutmap(bonds, ns)
    ks = syn.chain_ks(bonds, len(ns))
    E = [rng.standard_normal((4 ** k, 2 ** b)) for k, b in zip(ks, bits)]
    got = replay(plan_json(cm, out_bits=bits), E)
    ref = _einsum_chain(bonds, E)
    assert np.max(np.abs(got - ref)) < 1e-10 * max(1.0, np.abs(ref).max())


def _einsum_chain(bonds, E):
    """Eq. 1 for a chain written with explicit label axes (independent of the
    cut-map bookkeeping)."""
    import string
    letters = iter(string.ascii_letters)
    bond_letters = [[next(letters) for _ in range(b)] for b in bonds]
    terms, outs = [], []
    for c, e in enumerate(E):
        left = bond_letters[c - 1] if c > 0 else []
        right = bond_letters[c] if c < len(bonds) else []
        o = next(letters)
        outs.append(o)
        terms.append("".join(left + right) + o)
    ops = [e.reshape((4,) * (len(t) - 1) + (e.shape[1],)) for t, e in zip(terms, E)]
    K = sum(bonds)
    return np.einsum(",".join(terms) + "->" + "".join(outs), *ops).reshape(-1) * 2.0 ** -K


def test_plans_of_benchmark_workloads_need_no_permute():
    for bonds, ns in (([4, 4], [10, 10, 10]), ([3, 2, 3], [8, 8, 8, 8])):
        p = plan_json(syn.chain_cutmap(bonds, ns), "fp32")
        assert all(s["op"] == "gemm" for s in p["steps"])
        assert p["tensors"][p["steps"][-1]["c"]]["loc"] == "out"
    p = plan_json(syn.chain_cutmap([4, 4], [10, 10, 10]), "fp32")
    assert p["flops"] == pytest.approx(2 * (2 ** 10 * 2 ** 18 * 2 ** 8 + 2 ** 20 * 2 ** 10 * 2 ** 8))


def test_autotune_json_and_modes_without_gpu():
    import paper_2205_05836_amd as cq
    L = lib()
    need = C.c_size_t()
    assert L.cq_autotune_json(None, 0, C.byref(need)) == -1  # CQ_ERR_ARG: buffer too small
    assert need.value >= 3
    assert cq.cq_autotune_json() == []  # nothing tuned on a host without launches
    for mode in (0, 1, 2, 7, -3):
        assert L.cq_autotune_enable(mode) == 0
    cq.cq_autotune_enable(True)


def test_autotune_file_round_trip_without_gpu(tmp_path):
    """Tuned choices saved as text come back through cq_autotune_load with
    their schedule: lines of this kind of device are taken (without a GPU the
    device reads as "unknown"), lines of another device, of an unknown
    format or naming a variant that was not timed are skipped, and a file
    that does not exist is an error."""
    import paper_2205_05836_amd as cq
    ms = " ".join(["0.5"] * 12)
    good = f"cq-tune-1 unknown 3 1 0 1 0 1 1000003 1024 256 7 8 1023 {ms}\n"
    lines = [good,
             f"cq-tune-1 gfx942-304cu 3 1 0 1 0 1 1000005 1024 256 7 8 1023 {ms}\n",   # another device
             "not a tuning line\n",
             f"cq-tune-1 unknown 3 1 0 1 0 1 1000007 1024 256 7 9 255 {ms}\n"]         # 9 was not timed
    src = tmp_path / "tune.txt"
    src.write_text("".join(lines))
    cq.cq_autotune_load(str(src))
    got = [e for e in cq.cq_autotune_json() if e["M"] in (1000003, 1000005, 1000007)]
    assert len(got) == 1
    e = got[0]
    assert (e["prec"], e["N"], e["K"], e["Z"], e["variant"]) == ("bf16_split", 1024, 256, 7, 8)
    assert e["schedule"] == {"kernel": "occupancy", "tile": [128, 128], "ring": 2,
                             "workgroups_per_cu": 4, "raster": "default"}
    out = tmp_path / "saved.txt"
    cq.cq_autotune_save(str(out))
    assert good in out.read_text()
    with pytest.raises(cq.CQError) as err:
        cq.cq_autotune_load(str(tmp_path / "missing.txt"))
    assert err.value.status == -1


def test_plan_json_workspace_matches_fd_query():
    """The plan JSON reports the workspace cq_fd_workspace_size asks for, in
    every precision (the 16-bit forms include the per-label balance rows)."""
    import paper_2205_05836_amd as cq
    for bonds, ns in [([4, 4], [10, 10, 10]), ([3, 2, 3], [8, 8, 8, 8]), ([1], [3, 4])]:
        cm = syn.chain_cutmap(bonds, ns)
        for p in ("fp64", "fp32", "bf16", "bf16_split", "fp16", "fp16_split"):
            assert cq.cq_plan_json(cm, p)["workspace_bytes"] == cq.cq_fd_workspace_size(cm, p), (bonds, p)
