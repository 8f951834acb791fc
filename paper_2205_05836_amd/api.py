"""Thin Python binding of the C ABI (include/cutqc.h): argument marshalling
only.  torch provides device memory and the current stream; every step of the
reconstruction runs in the library's HIP kernels.

A subcircuit is a ``(width, init_cut, meas_cut)`` tuple or any object with
those attributes (see include/cutqc.h for the conventions).
"""
from __future__ import annotations

import ctypes as C
import os

from . import _lib
from ._lib import check, lib


def _sub_fields(sub):
    if isinstance(sub, (tuple, list)):
        w, ic, mc = sub
    else:
        w, ic, mc = sub.width, sub.init_cut, sub.meas_cut
    return int(w), [int(x) for x in ic], [int(x) for x in mc]


class _Subs:
    """Keeps the ctypes arrays of a subcircuit list alive for one call."""

    def __init__(self, subs):
        self.keep = []
        self.arr = (_lib.cq_subcircuit * len(subs))()
        self.n_out = []
        for i, s in enumerate(subs):
            w, ic, mc = _sub_fields(s)
            a = (C.c_int32 * max(w, 1))(*ic)
            b = (C.c_int32 * max(w, 1))(*mc)
            self.keep += [a, b]
            self.arr[i].width = w
            self.arr[i].init_cut = C.cast(a, C.POINTER(C.c_int32))
            self.arr[i].meas_cut = C.cast(b, C.POINTER(C.c_int32))
            self.n_out.append(sum(1 for m in mc if m == -1))

    def ptr(self, i=0):
        return C.cast(C.byref(self.arr, i * C.sizeof(_lib.cq_subcircuit)),
                      C.POINTER(_lib.cq_subcircuit))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype=None):
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _workspace(nbytes, device, workspace=None):
    import torch
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise ValueError("workspace too small")
        return workspace
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def cq_validate_cutmap(subs):
    """(K, n) of a cut map; raises CQError when it is inconsistent.  Host only."""
    s = _Subs(subs)
    k, n = C.c_int32(), C.c_int32()
    check(lib().cq_validate_cutmap(len(subs), s.ptr(), C.byref(k), C.byref(n)))
    return k.value, n.value


def cq_attribute_workspace_size(sub):
    s = _Subs([sub])
    b = C.c_size_t()
    check(lib().cq_attribute_workspace_size(s.ptr(), C.byref(b)))
    return b.value


def cq_attribute(sub, variants, entries=None, workspace=None, stream=None):
    """Entries (4^k, 2^n) FP64 of one subcircuit from its variant
    probabilities (4^r, 3^o, 2^w) FP64, both on the device."""
    import torch
    s = _Subs([sub])
    w, ic, mc = _sub_fields(sub)
    k = len({c for c in ic + mc if c != -1})
    n = s.n_out[0]
    if entries is None:
        entries = torch.empty((4 ** k, 2 ** n), dtype=torch.float64, device=variants.device)
    nbytes = cq_attribute_workspace_size(sub)
    ws = _workspace(nbytes, variants.device, workspace)
    check(lib().cq_attribute(s.ptr(), _dev_ptr(variants, torch.float64),
                             _dev_ptr(entries, torch.float64), _dev_ptr(ws), C.c_size_t(nbytes),
                             _stream(stream)))
    return entries


def _perm_arr(out_perm):
    if out_perm is None:
        return None
    return (C.c_int32 * len(out_perm))(*[int(q) for q in out_perm])


def cq_fd_workspace_size(subs, prec="fp64", out_perm=None):
    s = _Subs(subs)
    perm = _perm_arr(out_perm)
    b = C.c_size_t()
    check(lib().cq_fd_workspace_size(len(subs), s.ptr(), _lib.PRECISION[prec],
                                     C.cast(perm, C.POINTER(C.c_int32)) if perm else None,
                                     C.byref(b)))
    return b.value


def cq_reconstruct_fd(subs, entries, prec="fp64", out_perm=None, out=None, workspace=None,
                      stream=None):
    """Full-definition output (2^n) from FP64 device entries, one per
    subcircuit.  Returns float64 for prec='fp64', else float32."""
    import torch
    s = _Subs(subs)
    n = sum(s.n_out)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    dev = entries[0].device
    if out is None:
        out = torch.empty(2 ** n, dtype=dtype, device=dev)
    elif out.dtype != dtype or out.numel() != 2 ** n:
        raise ValueError("output tensor has the wrong dtype or size")
    perm = _perm_arr(out_perm)
    nbytes = cq_fd_workspace_size(subs, prec, out_perm)
    ws = _workspace(nbytes, dev, workspace)
    ptrs = (C.c_void_p * len(entries))(*[_dev_ptr(e, torch.float64).value for e in entries])
    check(lib().cq_reconstruct_fd(len(subs), s.ptr(), ptrs, _lib.PRECISION[prec],
                                  C.cast(perm, C.POINTER(C.c_int32)) if perm else None,
                                  _dev_ptr(out), _dev_ptr(ws), C.c_size_t(nbytes),
                                  _stream(stream)))
    return out


def cq_reconstruct_fd_noalloc(subs, entries, out, prec="fp64", out_perm=None, stream=None):
    """cq_reconstruct_fd on the library's fixed scratch (no workspace, no
    allocation inside the call).  ``out``: preallocated device tensor of 2^n
    values, float64 for prec='fp64' else float32."""
    import torch
    s = _Subs(subs)
    n = sum(s.n_out)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if out.dtype != dtype or out.numel() != 2 ** n:
        raise ValueError("output tensor has the wrong dtype or size")
    perm = _perm_arr(out_perm)
    ptrs = (C.c_void_p * len(entries))(*[_dev_ptr(e, torch.float64).value for e in entries])
    check(lib().cq_reconstruct_fd_noalloc(len(subs), s.ptr(), ptrs, _lib.PRECISION[prec],
                                          C.cast(perm, C.POINTER(C.c_int32)) if perm else None,
                                          _dev_ptr(out), _stream(stream)))
    return out


def _mask(positions):
    m = 0
    for p in positions:
        m |= 1 << int(p)
    return m


class _Instances:
    def __init__(self, instances):
        self.keep = []
        self.arr = (_lib.cq_dd_instance * len(instances))()
        for i, inst in enumerate(instances):
            subs = _Subs(inst["subs"])
            ns = len(inst["subs"])
            ptrs = (C.c_void_p * ns)(*[e.data_ptr() for e in inst["entries"]])
            act = (C.c_uint64 * ns)(*inst["active"])
            mer = (C.c_uint64 * ns)(*inst["merged"])
            fix = (C.c_uint64 * ns)(*inst.get("fixed", [0] * ns))
            fv = (C.c_uint64 * ns)(*inst.get("fixed_vals", [0] * ns))
            ma = (C.c_int32 * ns)(*inst["max_active"])
            self.keep += [subs, ptrs, act, mer, fix, fv, ma, inst["entries"]]
            a = self.arr[i]
            a.n_sub = ns
            a.subs = subs.ptr()
            a.entries = C.cast(ptrs, C.POINTER(C.c_void_p))
            a.active = C.cast(act, C.POINTER(C.c_uint64))
            a.merged = C.cast(mer, C.POINTER(C.c_uint64))
            a.fixed = C.cast(fix, C.POINTER(C.c_uint64))
            a.fixed_vals = C.cast(fv, C.POINTER(C.c_uint64))
            a.max_active = C.cast(ma, C.POINTER(C.c_int32))


def cq_dd_workspace_size(instances, prec="fp64", R=4, bins_stored=False):
    ins = _Instances(instances)
    par = _lib.cq_dd_params(_lib.PRECISION[prec], int(R), 0, 0, None, None)
    b = C.c_size_t()
    check(lib().cq_dd_workspace_size(len(instances), ins.arr, C.byref(par), int(bins_stored),
                                     C.byref(b)))
    return b.value


def cq_dd_checkpoint_bytes():
    """Bytes of one instance's dynamic-definition checkpoint."""
    return int(lib().cq_dd_checkpoint_bytes())


def cq_reconstruct_dd(instances, prec="fp64", R=4, bins=None, workspace=None, stream=None,
                      launch="graph", recursions=0, resume=None, checkpoint=False):
    """Dynamic definition over a batch of instances.  Each instance is a dict
    with keys subs, entries (FP64 device tensors), active, merged, fixed,
    fixed_vals (recursion-0 masks, bit i = output i, i = 0 most significant)
    and max_active.  ``bins``: optional list (instance-major, R per instance)
    of device tensors that receive each recursion's bins (each sized for the
    most bins a recursion can have).  ``launch``: "graph" (one hipGraph for
    the batch) or "direct".  ``recursions``: recursions this call runs per
    instance (0: up to R in total).  ``resume``: checkpoints (bytes) of an
    earlier call to continue from; ``checkpoint``: also return the states
    after this call.
    Returns (records, recursions_done), plus the checkpoints (bytes) when
    ``checkpoint``: records[i][j] is a dict for recursion
    records[i][j]["recursion"]."""
    ins = _Instances(instances)
    ck = cq_dd_checkpoint_bytes()
    res_buf = None
    if resume is not None:
        if len(resume) != ck * len(instances):
            raise ValueError("resume holds %d bytes, expected %d" % (len(resume), ck * len(instances)))
        res_buf = C.create_string_buffer(bytes(resume), len(resume))
    out_buf = C.create_string_buffer(ck * len(instances)) if checkpoint else None
    par = _lib.cq_dd_params(_lib.PRECISION[prec], int(R), _lib.DD_LAUNCH[launch], int(recursions),
                            C.cast(res_buf, C.c_void_p) if res_buf is not None else None,
                            C.cast(out_buf, C.c_void_p) if out_buf is not None else None)
    nbytes = cq_dd_workspace_size(instances, prec, R, bins is not None)
    dev = instances[0]["entries"][0].device
    ws = _workspace(nbytes, dev, workspace)
    recs = (_lib.cq_dd_record * (len(instances) * R))()
    done = (C.c_int32 * len(instances))()
    bin_ptrs = None
    if bins is not None:
        bin_ptrs = (C.c_void_p * (len(instances) * R))(
            *[(b.data_ptr() if b is not None else None) for b in bins])
    check(lib().cq_reconstruct_dd(len(instances), ins.arr, C.byref(par), recs,
                                  C.cast(bin_ptrs, C.POINTER(C.c_void_p)) if bin_ptrs else None,
                                  done, _dev_ptr(ws), C.c_size_t(nbytes), _stream(stream)))
    out = []
    for i, inst in enumerate(instances):
        ns = len(inst["subs"])
        rows = []
        for r in range(done[i]):
            rc = recs[i * R + r]
            rows.append(dict(
                recursion=rc.recursion, active=list(rc.active[:ns]), merged=list(rc.merged[:ns]),
                fixed=list(rc.fixed[:ns]), fixed_vals=list(rc.fixed_vals[:ns]),
                n_active=rc.n_active, total=rc.total,
                list=[(rc.list_val[j], rc.list_rec[j], rc.list_bin[j]) for j in range(rc.n_list)],
                popped=bool(rc.popped), tiles=rc.tiles, tiles_run=rc.tiles_run))
        out.append(rows)
    if checkpoint:
        return out, list(done), out_buf.raw
    return out, list(done)


def _record_dict(rc, ns):
    return dict(recursion=rc.recursion, active=list(rc.active[:ns]), merged=list(rc.merged[:ns]),
                fixed=list(rc.fixed[:ns]), fixed_vals=list(rc.fixed_vals[:ns]),
                n_active=rc.n_active, total=rc.total,
                list=[(rc.list_val[j], rc.list_rec[j], rc.list_bin[j]) for j in range(rc.n_list)],
                popped=bool(rc.popped), tiles=rc.tiles, tiles_run=rc.tiles_run)


def cq_dd_bfs_workspace_size(instance, prec="fp64", levels=2, width=4):
    ins = _Instances([instance])
    par = _lib.cq_dd_bfs_params(_lib.PRECISION[prec], int(levels), int(width), 0)
    b = C.c_size_t()
    check(lib().cq_dd_bfs_workspace_size(ins.arr, C.byref(par), C.byref(b)))
    return b.value


def cq_reconstruct_dd_bfs(instance, prec="fp64", levels=2, width=4, workspace=None, stream=None,
                          launch="graph"):
    """Breadth-first dynamic definition from one root instance (a dict as
    for cq_reconstruct_dd).  Returns the nodes in level order, each a dict:
    level, parent (node index, -1 for the root), parent_bin, and the
    node's record (masks, n_active, total, candidates in ``list``)."""
    ins = _Instances([instance])
    par = _lib.cq_dd_bfs_params(_lib.PRECISION[prec], int(levels), int(width),
                                _lib.DD_LAUNCH[launch])
    nbytes = cq_dd_bfs_workspace_size(instance, prec, levels, width)
    ws = _workspace(nbytes, instance["entries"][0].device, workspace)
    cap = max(1, 1 + (int(levels) - 1) * int(width))
    nodes = (_lib.cq_dd_bfs_node * cap)()
    n = C.c_int32()
    check(lib().cq_reconstruct_dd_bfs(ins.arr, C.byref(par), nodes, cap, C.byref(n), _dev_ptr(ws),
                                      C.c_size_t(nbytes), _stream(stream)))
    ns = len(instance["subs"])
    return [dict(level=nodes[k].level, parent=nodes[k].parent, parent_bin=nodes[k].parent_bin,
                 **_record_dict(nodes[k].rec, ns)) for k in range(n.value)]


def cq_sample_shots_workspace_size(rows, cols, shots):
    b = C.c_size_t()
    check(lib().cq_sample_shots_workspace_size(int(rows), int(cols), int(shots), C.byref(b)))
    return b.value


def cq_sample_shots(probs, shots, seed, out=None, workspace=None, stream=None):
    """Empirical frequencies of ``shots`` samples of every row of ``probs``
    (a device FP64 tensor, last axis = outcomes), as a new FP64 tensor of the
    same shape unless ``out`` is given."""
    import torch
    _dev_ptr(probs, torch.float64)
    cols = int(probs.shape[-1]) if probs.dim() else 1
    rows = probs.numel() // max(cols, 1)
    if out is None:
        out = torch.empty_like(probs)
    elif out.shape != probs.shape:
        raise ValueError("out must have the shape of probs")
    nbytes = cq_sample_shots_workspace_size(rows, cols, shots)
    ws = _workspace(nbytes, probs.device, workspace)
    check(lib().cq_sample_shots(_dev_ptr(probs), rows, cols, int(shots), C.c_uint64(int(seed)),
                                _dev_ptr(out, torch.float64), _dev_ptr(ws), C.c_size_t(nbytes),
                                _stream(stream)))
    return out


def cq_chi2_workspace_size():
    b = C.c_size_t()
    check(lib().cq_chi2_workspace_size(C.byref(b)))
    return b.value


def cq_chi2(a, b, out=None, workspace=None, stream=None):
    """Eq. 3 between two device FP64 tensors of equal size; returns a
    one-element device tensor (``out`` if given), written asynchronously."""
    import torch
    if a.numel() != b.numel():
        raise ValueError("a and b differ in size")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=a.device)
    nbytes = cq_chi2_workspace_size()
    ws = _workspace(nbytes, a.device, workspace)
    check(lib().cq_chi2(_dev_ptr(a, torch.float64), _dev_ptr(b, torch.float64), a.numel(),
                        _dev_ptr(out, torch.float64), _dev_ptr(ws), C.c_size_t(nbytes),
                        _stream(stream)))
    return out


def _gates(ops):
    """Gate list -> ctypes array.  An op is an object with ``name`` ('u' or
    'cz'), ``qubits`` and ``matrix`` (2 x 2 complex for 'u'), or a tuple
    ('u', q, matrix) / ('cz', q0, q1)."""
    ops = list(ops)
    arr = (_lib.cq_gate * max(len(ops), 1))()
    for i, op in enumerate(ops):
        if isinstance(op, tuple):
            name, rest = op[0], op[1:]
            qubits = (rest[0],) if name == "u" else (rest[0], rest[1])
            matrix = rest[1] if name == "u" else None
        else:
            name, qubits, matrix = op.name, op.qubits, op.matrix
        if name == "u":
            arr[i].kind, arr[i].q0 = _lib.GATE_U, int(qubits[0])
            m = [complex(matrix[r][c]) for r in range(2) for c in range(2)]
            for j, z in enumerate(m):
                arr[i].u[2 * j], arr[i].u[2 * j + 1] = z.real, z.imag
        elif name == "cz":
            arr[i].kind, arr[i].q0, arr[i].q1 = _lib.GATE_CZ, int(qubits[0]), int(qubits[1])
        else:
            raise ValueError(f"unknown gate {name!r}")
    return arr, len(ops)


def cq_simulate_workspace_size(n):
    b = C.c_size_t()
    check(lib().cq_simulate_workspace_size(int(n), C.byref(b)))
    return b.value


def cq_simulate_probabilities(n, ops, out=None, workspace=None, device="cuda:0", stream=None):
    """|psi|^2 (2^n FP64 on the device) of ``ops`` applied to |0...0>."""
    import torch
    if out is None:
        out = torch.empty(2 ** int(n), dtype=torch.float64, device=device)
    elif out.numel() != 2 ** int(n):
        raise ValueError("out must hold 2^n values")
    arr, cnt = _gates(ops)
    nbytes = cq_simulate_workspace_size(n)
    ws = _workspace(nbytes, out.device, workspace)
    check(lib().cq_simulate_probabilities(int(n), arr, cnt, _dev_ptr(out, torch.float64), _dev_ptr(ws),
                                          C.c_size_t(nbytes), _stream(stream)))
    return out


def cq_variants_workspace_size(sub):
    s = _Subs([sub])
    b = C.c_size_t()
    check(lib().cq_variants_workspace_size(s.ptr(), C.byref(b)))
    return b.value


def cq_variant_probabilities(sub, ops=None, out=None, workspace=None, device="cuda:0", stream=None):
    """Every variant of subcircuit ``sub`` (its ``ops`` unless given) as a
    (4^r, 3^o, 2^width) FP64 device tensor, the layout cq_attribute reads."""
    import torch
    w, ic, mc = _sub_fields(sub)
    if ops is None:
        if not hasattr(sub, "ops"):
            raise ValueError("pass ops for a subcircuit given as a tuple")
        ops = sub.ops
    r = sum(1 for x in ic if x != -1)
    o = sum(1 for x in mc if x != -1)
    shape = (4 ** r, 3 ** o, 2 ** w)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=device)
    elif tuple(out.shape) != shape:
        raise ValueError(f"out must have shape {shape}")
    s = _Subs([sub])
    arr, cnt = _gates(ops)
    nbytes = cq_variants_workspace_size(sub)
    ws = _workspace(nbytes, out.device, workspace)
    check(lib().cq_variant_probabilities(s.ptr(), arr, cnt, _dev_ptr(out, torch.float64), _dev_ptr(ws),
                                         C.c_size_t(nbytes), _stream(stream)))
    return out


def cq_find_cuts(n_qubits, gates, max_width, max_subcircuits=5):
    """Exact minimum-cost clustering of a small circuit's two-qubit gates
    (host only).  ``gates``: qubit pairs in circuit order, or ops whose
    two-qubit ones ('cz') are taken.  Returns a dict with each gate's
    ``cluster``, ``n_subcircuits``, ``n_cuts`` and ``cost``."""
    pairs = []
    for g in gates:
        if isinstance(g, (tuple, list)):
            pairs.append((int(g[0]), int(g[1])))
        elif len(g.qubits) == 2:
            pairs.append((int(g.qubits[0]), int(g.qubits[1])))
    flat = (C.c_int32 * max(2 * len(pairs), 1))(*[q for p in pairs for q in p])
    prob = _lib.cq_cut_problem(int(n_qubits), len(pairs), C.cast(flat, C.POINTER(C.c_int32)),
                               int(max_width), int(max_subcircuits))
    cluster = (C.c_int32 * max(len(pairs), 1))()
    ns, nc, cost = C.c_int32(), C.c_int32(), C.c_double()
    check(lib().cq_find_cuts(C.byref(prob), cluster, C.byref(ns), C.byref(nc), C.byref(cost)))
    return dict(cluster=list(cluster[:len(pairs)]), n_subcircuits=ns.value, n_cuts=nc.value,
                cost=cost.value)


def cq_plan_json(subs, prec="fp64", out_bits=None, out_perm=None):
    """The contraction plan as a dict (host only, launches nothing)."""
    import json
    s = _Subs(subs)
    ob = (C.c_int32 * len(subs))(*out_bits) if out_bits is not None else None
    op = _perm_arr(out_perm)
    need = C.c_size_t()
    lib().cq_plan_json(len(subs), s.ptr(), _lib.PRECISION[prec], ob, op, None, 0, C.byref(need))
    buf = C.create_string_buffer(need.value)
    check(lib().cq_plan_json(len(subs), s.ptr(), _lib.PRECISION[prec], ob, op, buf, need.value,
                             C.byref(need)))
    return json.loads(buf.value.decode())


def cq_autotune_enable(on=True, variant=None):
    """Turn GEMM autotuning on or off; ``variant=v`` forces variant v."""
    mode = 2 + int(variant) if variant is not None else (1 if on else 0)
    check(lib().cq_autotune_enable(mode))


def cq_label_balance_enable(mode=1):
    """Per-label balance of the 16-bit operands: 0 off, 1 FP16 forms
    (default), 2 every 16-bit form."""
    check(lib().cq_label_balance_enable(int(mode)))


def cq_column_scaling_enable(on=True):
    """Column scaling of the FP16 and FP16-split operands (FD and DD): on by
    default.  Query workspace sizes after changing it."""
    check(lib().cq_column_scaling_enable(1 if on else 0))


def cq_dd_lanes(lanes=0):
    """Parallel lanes of cq_reconstruct_dd (0: the default, 4; at most 8).
    Query the workspace size after changing it."""
    check(lib().cq_dd_lanes(int(lanes)))


def cq_autotune_load(path):
    """Add the tuned choices saved in `path` (this kind of device's) to the cache."""
    check(lib().cq_autotune_load(os.fsencode(path)))


def cq_autotune_save(path):
    """Write the cached tuned choices to `path`."""
    check(lib().cq_autotune_save(os.fsencode(path)))


def cq_autotune_json():
    """The autotuner's cached choices (list of dicts)."""
    import json
    need = C.c_size_t()
    lib().cq_autotune_json(None, 0, C.byref(need))
    buf = C.create_string_buffer(need.value)
    check(lib().cq_autotune_json(buf, need.value, C.byref(need)))
    return json.loads(buf.value.decode())


def cq_profile_enable(on=True):
    check(lib().cq_profile_enable(1 if on else 0))


def cq_profile_read(cap=65536):
    """[(kernel name, milliseconds, flops)] of the launches since the last read."""
    names = C.create_string_buffer(32 * cap)
    ms = (C.c_double * cap)()
    fl = (C.c_double * cap)()
    cnt = C.c_int32()
    check(lib().cq_profile_read(names, ms, fl, cap, C.byref(cnt)))
    raw = names.raw
    return [(raw[32 * i:32 * i + 32].split(b"\0")[0].decode(), ms[i], fl[i])
            for i in range(min(cnt.value, cap))]


# Friendlier aliases
attribute = cq_attribute
reconstruct_fd = cq_reconstruct_fd
reconstruct_dd = cq_reconstruct_dd
validate_cutmap = cq_validate_cutmap
mask = _mask
