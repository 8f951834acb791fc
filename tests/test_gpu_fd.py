"""GPU parity of entry attribution and full-definition reconstruction against
the FP64 oracle, through the C ABI.

Tolerances: the FP64 path must match the oracle within 1e-10 max-abs;
integer-valued entries make every sum exact, so there the GPU must match
bit for bit (FP64 and FP32); the FP32 path on Dirichlet/uniform data must stay
within 1e-6 max-abs.

Because the Dirichlet(0.1) workloads put most bins at tiny values, each check
also bounds the error relative to the bin's rounding scale
2^-K sum_l prod_c |E_c[l, b_c]|: 1e-13 for FP64, 1e-5 for FP32.  FP32 has no
normal numbers below 2^-126, so the FP32 bounds carry the absolute floor
fp32_floor(cut map) derived below (about 1e-32 at K = 8) for bins whose terms
underflow."""
import numpy as np
import pytest

from oracle import attribution as at
from oracle import cutmap
from oracle import reconstruct as rc
from oracle import statevector as sv
from workloads import circuits as wc
from workloads import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def fp32_floor(cm):
    """Absolute error below FP32's normal range for operands of magnitude at
    most 1 (every synthetic entry is bounded by its identity row, a Dirichlet
    draw).  Each elementary step -- the conversion of an operand, a product,
    an addition, the final scaling -- whose result falls below 2^-126 adds at
    most 2^-126.  The output is a sum of 4^K label terms of n_C factors, a
    term passes through at most 3 n_C + 1 such steps, and an error injected at
    a step reaches the output multiplied by at most the number of terms that
    use it (the other factors and 2^-K are at most 1 in magnitude), so the
    total is at most (3 n_C + 1) 4^K 2^-126."""
    return (3 * len(cm) + 1) * 4.0 ** cutmap.total_cuts(cm) * 2.0 ** -126


def cq():
    import paper_2205_05836_amd as m
    return m


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def gpu_attribute(spec, V):
    return cq().cq_attribute(spec, to_dev(V)).cpu().numpy()


def gpu_fd(subs, ents, prec, out_perm=None):
    out = cq().cq_reconstruct_fd(subs, [to_dev(e) for e in ents], prec=prec, out_perm=out_perm)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("which", ["8q", "20q"])
def test_circuit_attribution_and_fd_match_oracle_and_statevector(which):
    cc = wc.two_way_circuit_8q(0) if which == "8q" else wc.two_way_circuit_20q(1)
    print(f"case {which}", flush=True)
    subs = cc.subcircuits()
    Vs = [sv.variant_probabilities(s) for s in subs]
    E_or = [at.attribute(s, V) for s, V in zip(subs, Vs)]
    E_gpu = [gpu_attribute(s, V) for s, V in zip(subs, Vs)]
    for a, b in zip(E_gpu, E_or):
        assert a.shape == b.shape
        assert np.max(np.abs(a - b)) < 1e-13
    p_or = rc.apply_out_perm(rc.fd_contract(subs, E_or), cc.out_perm())
    p_sv = sv.probabilities(cc.n_qubits, cc.ops)
    p64 = gpu_fd(subs, E_gpu, "fp64", cc.out_perm())
    assert np.max(np.abs(p64 - p_or)) < 1e-10
    assert np.max(np.abs(p64 - p_sv)) < 1e-10
    p32 = gpu_fd(subs, E_gpu, "fp32", cc.out_perm())
    assert np.max(np.abs(p32 - p_or)) < 1e-6


def _random_circuits(count, seed0=900):
    out, seed = [], seed0
    while len(out) < count:
        rng = np.random.default_rng(seed)
        seed += 1
        cc = wc.random_cut_circuit(rng, int(rng.integers(4, 9)), int(rng.integers(2, 4)),
                                   int(rng.integers(1, 4)), depth=5)
        if cc is None or not cc.cuts:
            continue
        if sum(len(cutmap.outputs(s)) for s in cc.subcircuits()) != cc.n_qubits:
            continue
        out.append(cc)
    return out


@pytest.mark.parametrize("idx", range(8))
def test_random_cut_circuits(idx):
    cc = _random_circuits(8)[idx]
    subs = cc.subcircuits()
    print(f"random circuit {idx}: n={cc.n_qubits} subs={len(subs)} cuts={len(cc.cuts)}", flush=True)
    Vs = [sv.variant_probabilities(s) for s in subs]
    E_gpu = [gpu_attribute(s, V) for s, V in zip(subs, Vs)]
    E_or = [at.attribute(s, V) for s, V in zip(subs, Vs)]
    for a, b in zip(E_gpu, E_or):
        assert np.max(np.abs(a - b)) < 1e-13
    p_sv = sv.probabilities(cc.n_qubits, cc.ops)
    p64 = gpu_fd(subs, E_gpu, "fp64", cc.out_perm())
    assert np.max(np.abs(p64 - p_sv)) < 1e-10


INT_CASES = [
    ([2, 1], [3, 5, 7]),       # ragged tiles everywhere
    ([1, 2], [7, 6, 7]),       # 2^20 outputs, several tiles
    ([3], [9, 8]),             # two subcircuits
    ([0, 2], [4, 4, 5]),       # a bond without cuts: outer product
    ([2, 1, 2], [4, 3, 4, 5]), # chain of four
    ([2], [0, 6]),             # a subcircuit without outputs
]


@pytest.mark.parametrize("bonds,ns", INT_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_integer_entries_bit_exact(bonds, ns, prec):
    print(f"int case bonds={bonds} ns={ns} {prec}", flush=True)
    rng = np.random.default_rng(sum(ns) * 7 + len(bonds))
    cm = syn.chain_cutmap(bonds, ns)
    ks = syn.chain_ks(bonds, len(ns))
    E = [syn.integer_entries(rng, k, n, lo=-4, hi=4) for k, n in zip(ks, ns)]
    ref = rc.fd_contract(cm, E)
    got = gpu_fd(cm, E, prec)
    assert np.array_equal(got, ref)


def test_single_subcircuit_no_cuts():
    rng = np.random.default_rng(3)
    E = [rng.standard_normal((1, 2 ** 11))]
    cm = [(11, [-1] * 11, [-1] * 11)]
    assert np.array_equal(gpu_fd(cm, E, "fp64"), E[0][0])
    perm = list(rng.permutation(11))
    assert np.array_equal(gpu_fd(cm, E, "fp64", perm), rc.apply_out_perm(E[0][0], perm))


def test_out_perm_bit_exact_on_chain():
    rng = np.random.default_rng(5)
    cm = syn.chain_cutmap([2, 1], [5, 4, 6])
    E = [syn.integer_entries(rng, k, n) for k, n in zip(syn.chain_ks([2, 1], 3), [5, 4, 6])]
    perm = [int(x) for x in rng.permutation(15)]
    ref = rc.apply_out_perm(rc.fd_contract(cm, E), perm)
    for prec in ("fp64", "fp32"):
        assert np.array_equal(gpu_fd(cm, E, prec, perm), ref)


def test_dirichlet_chain_fp64_and_fp32():
    cm, E = syn.chain_instance(12, [3, 2], [8, 6, 7])
    ref = rc.fd_contract(cm, E)
    scale = rc.fd_contract(cm, [np.abs(e) for e in E])
    e64 = np.abs(gpu_fd(cm, E, "fp64") - ref)
    e32 = np.abs(gpu_fd(cm, E, "fp32") - ref)
    assert e64.max() < 1e-10 and np.max(e64 / scale) < 1e-13
    assert e32.max() < 1e-6 and np.all(e32 <= 1e-5 * scale + fp32_floor(cm))


def test_deterministic_repeat():
    cm, E = syn.chain_instance(13, [4, 4], [8, 8, 8])
    a = gpu_fd(cm, E, "fp32")
    b = gpu_fd(cm, E, "fp32")
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec,variants", [("fp64", 2), ("fp32", 12), ("bf16_split", 12),
                                            ("fp16", 12), ("fp16_split", 12), ("bf16", 12)])
def test_every_gemm_variant_matches_oracle(prec, variants):
    """Each autotuner variant forced in turn; 2^24 outputs give every GEMM
    hundreds of tiles, so all variants apply.  Raster order changes no sum,
    so the two rasters of one implementation agree bit for bit.  In the FP16
    forms the last GEMM also applies the column-scaling exponents in its
    epilogue; every implementation computes the same products in the same
    order and applies them the same way, so all variants agree bit for
    bit."""
    m = cq()
    cm, E = syn.chain_instance(14, [4, 4], [8, 8, 8])
    ref = rc.fd_contract(cm, E)
    scale = rc.fd_contract(cm, [np.abs(e) for e in E])
    tol = {"fp64": 1e-13, "fp32": 1e-5, **H16_REL}[prec]
    outs = []
    try:
        for v in range(variants):
            m.cq_autotune_enable(variant=v)
            print(f"{prec} variant {v}", flush=True)
            out = gpu_fd(cm, E, prec)
            err = np.abs(out - ref)
            assert np.all(err <= tol * scale + fp32_floor(cm)), (prec, v, float(err.max()))
            outs.append(out)
        for v in range(0, variants, 2):
            assert np.array_equal(outs[v], outs[v + 1]), (prec, v)
        if prec in ("fp16", "fp16_split"):
            for v in range(variants):
                assert np.array_equal(outs[v], outs[0]), (prec, v)
        m.cq_autotune_enable(True)
        tuned = gpu_fd(cm, E, prec)
        again = gpu_fd(cm, E, prec)
        assert np.array_equal(tuned, again)
        assert any(np.array_equal(tuned, o) for o in outs)
        shapes = [e for e in m.cq_autotune_json() if e["prec"] == prec]
        assert shapes and all(0 <= e["variant"] < variants for e in shapes)
    finally:
        m.cq_autotune_enable(True)


# final GEMMs with ragged tiles (M or N below 128) and 8192 tiles, so every
# workgroup of the persistent kernel takes many tiles; K = 256, 64 and 16
RAGGED = [(22, [4, 4], [10, 4, 10]), (23, [3, 3], [10, 3, 10]), (24, [5, 2], [10, 10, 4])]


@pytest.mark.parametrize("seed,bonds,ns", RAGGED)
@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16_split"])
def test_persistent_gemm_ragged_tiles(seed, bonds, ns, prec):
    """Variant 2 (FP32: 64 x 64 tiles; 16-bit: the other ring depth),
    variant 4 (16-bit: 64 x 64 tiles), variants 6 and 7 (persistent kernel,
    both rasters) and 8 and 10 (the
    occupancy kernels: for the 16-bit forms two- and three-deep rings, for
    FP32 three- and four-deep rings) against variant 0 bit for bit -- same
    products, same order -- and against the oracle."""
    m = cq()
    cm, E = syn.chain_instance(seed, bonds, ns)
    ref = rc.fd_contract(cm, E)
    scale = rc.fd_contract(cm, [np.abs(e) for e in E])
    outs = {}
    try:
        for v in (0, 2, 4, 6, 7, 8, 10):
            m.cq_autotune_enable(variant=v)
            print(f"{prec} {bonds} {ns} variant {v}", flush=True)
            outs[v] = gpu_fd(cm, E, prec)
    finally:
        m.cq_autotune_enable(True)
    err = np.abs(outs[0] - ref)
    assert np.all(err <= {"fp32": 1e-5, **H16_REL}[prec] * scale + fp32_floor(cm)), float(err.max())
    for v in (2, 4, 6, 7, 8, 10):
        assert np.array_equal(outs[v], outs[0]), v


def test_workspace_too_small_writes_nothing():
    m = cq()
    cm, E = syn.chain_instance(14, [4, 4], [6, 6, 6])
    need = m.cq_fd_workspace_size(cm, "fp32")
    assert need > 0
    out = torch.full((2 ** 18,), 7.0, dtype=torch.float32, device=DEV)
    ws = torch.empty(need - 256, dtype=torch.uint8, device=DEV)
    import ctypes as C
    from paper_2205_05836_amd import _lib
    from paper_2205_05836_amd.api import _Subs, _dev_ptr, _stream
    s = _Subs(cm)
    ents = [to_dev(e) for e in E]
    ptrs = (C.c_void_p * 3)(*[e.data_ptr() for e in ents])
    st = _lib.lib().cq_reconstruct_fd(3, s.ptr(), ptrs, 1, None, _dev_ptr(out), _dev_ptr(ws),
                                      C.c_size_t(need - 256), _stream(None))
    torch.cuda.synchronize()
    assert st == -5
    assert bool(torch.all(out == 7.0))


# --- the 30-qubit, three-subcircuit workload at full size ------------------

SEED_30Q = 2
BONDS_30Q = [4, 4]
NS_30Q = [10, 10, 10]


def _entries_30q():
    ks = syn.chain_ks(BONDS_30Q, 3)
    return [syn.entries_torch(SEED_30Q, c, ks[c], NS_30Q[c], DEV) for c in range(3)]


def _sampled_reference(bins, absolute=False):
    """Oracle values at the sampled bins (or, with ``absolute``, the error
    scale 2^-K sum_l prod_c |E_c[l, b_c]| of each bin).  The needed entry columns are rebuilt
    on the host from the counter-based generator; sample j's columns are
    placed in column j of small local entry tensors, and the per-bin oracle is
    asked for the bin whose three parts all equal j."""
    cm = syn.chain_cutmap(BONDS_30Q, NS_30Q)
    ks = syn.chain_ks(BONDS_30Q, 3)
    parts = [(bins >> 20) & 1023, (bins >> 10) & 1023, bins & 1023]
    assert len(bins) <= 1024
    local = []
    for c in range(3):
        e = np.zeros((4 ** ks[c], 1024))
        e[:, :len(bins)] = syn.entries_columns(SEED_30Q, c, ks[c], 10, parts[c])
        local.append(np.abs(e) if absolute else e)
    j = np.arange(len(bins), dtype=np.int64)
    return rc.fd_per_bin(cm, local, (j << 20) | (j << 10) | j)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-6)])
def test_30_qubit_chain_full_size_sampled(prec, tol):
    m = cq()
    cm = syn.chain_cutmap(BONDS_30Q, NS_30Q)
    ents = _entries_30q()
    print(f"30q full size {prec}", flush=True)
    out = m.cq_reconstruct_fd(cm, ents, prec=prec)
    torch.cuda.synchronize()
    rng = np.random.default_rng(31)
    # uniform samples, the corners, and the heaviest bins (largest identity rows)
    heavy = [np.argsort(syn.identity_row(SEED_30Q, c, 10))[-4:] for c in range(3)]
    hb = [(a << 20) | (b << 10) | c for a in heavy[0] for b in heavy[1] for c in heavy[2]]
    bins = np.concatenate([rng.integers(0, 2 ** 30, size=900), hb,
                           [0, 2 ** 30 - 1, 1023, 2 ** 20, 2 ** 30 - 1024]]).astype(np.int64)
    got = out[torch.from_numpy(bins).to(DEV)].cpu().numpy().astype(np.float64)
    ref = _sampled_reference(bins)
    scale = _sampled_reference(bins, absolute=True)
    err = np.abs(got - ref)
    print(f"max abs err {err.max():.3e}, max |p| {np.abs(ref).max():.3e}, "
          f"max err/scale {np.max(err / scale):.3e}", flush=True)
    assert err.max() < tol
    # error relative to the rounding scale of each bin
    if prec == "fp64":
        assert np.max(err / scale) < 1e-13
    else:
        assert np.all(err <= 1e-5 * scale + fp32_floor(cm))
    # closed form of the total (sum over all bins): 2^-K sum_l prod_c rowsum_c(l_c),
    # row sums of the host-built entries contracted by the oracle
    ks = syn.chain_ks(BONDS_30Q, 3)
    rs = [syn.dirichlet_entries(SEED_30Q, c, ks[c], 10).sum(axis=1)[:, None] for c in range(3)]
    tot = float(rc.fd_contract(cm, rs)[0])
    got_tot = float(torch.sum(out, dtype=torch.float64).item())
    assert abs(got_tot - tot) < (1e-9 if prec == "fp64" else 1e-4)


# --- 16-bit matrix-core forms ------------------------------------------------

# Relative-to-scale bounds: one rounding of each operand to 8 significant bits
# (BF16) or 11 (FP16) plus FP32 accumulation; the split forms keep 16 / 22
# bits of each operand and drop only lo*lo.
H16_REL = {"bf16": 3e-2, "bf16_split": 3e-4, "fp16": 4e-3, "fp16_split": 1e-5}


@pytest.mark.parametrize("prec", ["bf16_split", "fp16", "fp16_split"])
@pytest.mark.parametrize("bonds,ns", [([2, 1], [3, 5, 7]), ([1, 2], [7, 6, 7]), ([3], [9, 8])])
def test_h16_integer_entries_exact(bonds, ns, prec):
    # integer entries in [-4, 4] need no low part; every intermediate stays an
    # integer below 2^11 (FP16) or is carried exactly by hi + lo (split forms)
    print(f"h16 int case bonds={bonds} ns={ns} {prec}", flush=True)
    rng = np.random.default_rng(sum(ns) * 7 + len(bonds))
    cm = syn.chain_cutmap(bonds, ns)
    ks = syn.chain_ks(bonds, len(ns))
    E = [syn.integer_entries(rng, k, n, lo=-4, hi=4) for k, n in zip(ks, ns)]
    ref = rc.fd_contract(cm, E)
    if prec == "fp16" and np.abs(ref).max() * 2 ** sum(bonds) >= 2048:
        pytest.skip("intermediate exceeds the FP16 integer range")
    got = gpu_fd(cm, E, prec)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("prec", ["bf16", "bf16_split"])
def test_h16_dirichlet_chain(prec):
    cm, E = syn.chain_instance(12, [3, 2], [8, 6, 7])
    ref = rc.fd_contract(cm, E)
    scale = rc.fd_contract(cm, [np.abs(e) for e in E])
    err = np.abs(gpu_fd(cm, E, prec) - ref)
    print(f"{prec}: max abs {err.max():.3e}")
    # plain BF16 keeps 8 significant bits: on this small chain (2^21 outputs,
    # probabilities up to ~1e-3) it cannot reach 1e-6; only its rounding bound
    # is asserted.  The split form must meet 1e-6.
    if prec == "bf16_split":
        assert err.max() < 1e-6
    assert np.all(err <= H16_REL[prec] * scale + fp32_floor(cm))


@pytest.mark.parametrize("prec", ["fp16", "fp16_split"])
def test_fp16_column_scaling_on_imbalanced_columns(prec):
    """Entry columns scaled down by 2^-6 (2^-5) per set output bit, so bins
    span about 2^-70: with the column scaling every bin stays within the
    FP16 rounding bound relative to its own magnitude (the bins of |E|);
    without it the small columns underflow FP16 and that bound fails."""
    m = cq()
    cm, E = syn.chain_instance(13, [2, 2], [7, 6, 7])
    E = [np.ldexp(e, -s * np.array([bin(b).count("1") for b in range(e.shape[1])])[None, :])
         for s, e in zip([0, 6, 5], E)]
    ref = rc.fd_contract(cm, E)
    scale = rc.fd_contract(cm, [np.abs(e) for e in E])
    bound = H16_REL[prec] * scale + fp32_floor(cm)
    got = gpu_fd(cm, E, prec)
    try:
        m.cq_column_scaling_enable(False)
        got_off = gpu_fd(cm, E, prec)
    finally:
        m.cq_column_scaling_enable(True)
    r_on = np.max(np.abs(got - ref) / bound)
    r_off = np.max(np.abs(got_off - ref) / bound)
    print(f"{prec}: max err / bound {r_on:.3e}, without column scaling {r_off:.3e}", flush=True)
    assert r_on <= 1.0
    assert not r_off <= 1.0   # lost small bins (or nan) without it


def test_h16_chain_of_four_split():
    cm, E = syn.chain_instance(15, [2, 1, 2], [5, 4, 5, 5])
    ref = rc.fd_contract(cm, E)
    scale = rc.fd_contract(cm, [np.abs(e) for e in E])
    err = np.abs(gpu_fd(cm, E, "bf16_split") - ref)
    assert np.all(err <= H16_REL["bf16_split"] * scale + fp32_floor(cm))


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
def test_30_qubit_chain_variants_bit_equal(prec):
    """At the benchmark shape every GEMM variant -- one tile per workgroup,
    flipped raster, persistent -- gives the same 2^30 outputs bit for bit
    (same products, same order), so the autotuner's choice never changes a
    result."""
    m = cq()
    cm = syn.chain_cutmap(BONDS_30Q, NS_30Q)
    ents = _entries_30q()
    ref = None
    try:
        for v in (0, 1, 6, 7, 8, 9, 10, 11):
            m.cq_autotune_enable(variant=v)
            print(f"30q {prec} variant {v}", flush=True)
            out = m.cq_reconstruct_fd(cm, ents, prec=prec)
            torch.cuda.synchronize()
            if ref is None:
                ref = out
            else:
                assert torch.equal(out, ref), (prec, v)
                del out
    finally:
        m.cq_autotune_enable(True)


@pytest.mark.parametrize("prec", ["bf16", "bf16_split", "fp16", "fp16_split"])
def test_30_qubit_chain_full_size_h16(prec):
    """Sampled and heaviest bins of the 30-qubit chain against the oracle in
    every 16-bit form; the FP16 forms run with the per-label balance and the
    column scaling, their last GEMM applying the exponents in its epilogue."""
    m = cq()
    cm = syn.chain_cutmap(BONDS_30Q, NS_30Q)
    ents = _entries_30q()
    print(f"30q full size {prec}", flush=True)
    out = m.cq_reconstruct_fd(cm, ents, prec=prec)
    torch.cuda.synchronize()
    rng = np.random.default_rng(32)
    heavy = [np.argsort(syn.identity_row(SEED_30Q, c, 10))[-4:] for c in range(3)]
    hb = [(a << 20) | (b << 10) | c for a in heavy[0] for b in heavy[1] for c in heavy[2]]
    bins = np.concatenate([rng.integers(0, 2 ** 30, size=900), hb]).astype(np.int64)
    got = out[torch.from_numpy(bins).to(DEV)].cpu().numpy().astype(np.float64)
    ref = _sampled_reference(bins)
    scale = _sampled_reference(bins, absolute=True)
    err = np.abs(got - ref)
    print(f"max abs err {err.max():.3e}, max err/scale {np.max(err / scale):.3e}", flush=True)
    assert err.max() < 1e-6
    assert np.all(err <= H16_REL[prec] * scale + fp32_floor(cm))


# --- per-label balance of the 16-bit operands --------------------------------

LABEL_SHIFT = {0: 0, 1: 20, 2: -20, 3: 10}   # digit I, X, Y, Z -> log2 factor


def imbalance_labels(cm, E, shift=LABEL_SHIFT):
    """Entries whose rows are scaled per cut label: a row with digit d at cut
    j gets 2^shift[d] on the subcircuit measuring j and 2^-shift[d] on the one
    initialising it.  Every labelling term of Eq. 1 keeps its value exactly,
    so the reconstruction is unchanged, but within one subcircuit the label
    rows now differ by up to 2^40."""
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


def test_label_balance_keeps_bf16_bits():
    """For the BF16 forms a power of two changes no rounding while values stay
    in BF16's normal range (FP32's exponents): balanced and unbalanced runs
    agree bit for bit.  Entries here are in +-[1e-3, 1], so even the 2^+-100
    row factors keep every operand and product normal (Dirichlet entries reach
    below 1e-38, where scaling does change what underflows)."""
    m = cq()
    rng = np.random.default_rng(12)
    cm = syn.chain_cutmap([3, 2], [8, 6, 7])
    E = [np.copysign(rng.uniform(1e-3, 1.0, size=(4 ** k, 2 ** n)), rng.uniform(-1, 1, size=(4 ** k, 2 ** n)))
         for k, n in zip(syn.chain_ks([3, 2], 3), [8, 6, 7])]
    Ei = imbalance_labels(cm, E)
    try:
        for prec in ("bf16", "bf16_split"):
            m.cq_label_balance_enable(0)
            off = gpu_fd(cm, Ei, prec)
            m.cq_label_balance_enable(2)
            on = gpu_fd(cm, Ei, prec)
            assert np.array_equal(on, off), prec
    finally:
        m.cq_label_balance_enable(1)


@pytest.mark.parametrize("bonds,ns", [([3, 2], [8, 6, 7]), ([4, 4], [6, 4, 6])])
@pytest.mark.parametrize("prec", ["fp16", "fp16_split"])
def test_label_balance_rescues_fp16_on_imbalanced_labels(prec, bonds, ns):
    """Label rows 2^+-20 apart within a subcircuit: without the balance the
    FP16 conversion loses the small rows (column scaling cannot help, the
    rows share columns); with it both sides of every cut meet in FP16's
    range and the result matches the oracle as on balanced data.  The second
    shape has 4^8 label rows in the middle subcircuit, so four of its digit
    positions lie above the balance kernel's 256-row stride."""
    m = cq()
    cm, E = syn.chain_instance(12, bonds, ns)
    Ei = imbalance_labels(cm, E)
    ref = rc.fd_contract(cm, E)
    assert np.array_equal(rc.fd_contract(cm, Ei), ref)  # the input change is exact
    scale = rc.fd_contract(cm, [np.abs(e) for e in E])
    try:
        m.cq_label_balance_enable(0)
        err_off = np.abs(gpu_fd(cm, Ei, prec) - ref)
        m.cq_label_balance_enable(1)
        err_on = np.abs(gpu_fd(cm, Ei, prec) - ref)
        err_plain = np.abs(gpu_fd(cm, E, prec) - ref)
    finally:
        m.cq_label_balance_enable(1)
    print(f"{prec}: max abs balanced input {err_plain.max():.3e}; imbalanced without balance "
          f"{err_off.max():.3e}, with balance {err_on.max():.3e}", flush=True)
    tol = {"fp16": 4e-3, "fp16_split": 1e-5}[prec]
    assert np.all(err_on <= tol * scale + fp32_floor(cm))
    assert err_on.max() <= 4 * err_plain.max() + 1e-30
    if prec == "fp16_split":
        assert err_on.max() < 1e-6
    # the arm matters: without the balance the error is far larger
    assert err_off.max() > 100 * err_on.max()


# --- 32-qubit chain of four: the mixed-precision accuracy matrix -------------

SEED_32Q = 3
BONDS_32Q = [3, 2, 3]        # K = 8; label rows 64, 1024, 1024, 64
NS_32Q = [8, 8, 8, 8]        # 2^32 outputs


def _full_vs(out, ref_out, chunk=1 << 27):
    """max |a - b| and total variation over all outputs (device, float64)."""
    mx, tv = 0.0, 0.0
    for i in range(0, out.numel(), chunk):
        d = (out[i:i + chunk].double() - ref_out[i:i + chunk].double()).abs()
        mx = max(mx, float(d.max()))
        tv += float(d.sum())
    return mx, 0.5 * tv


_FP64_32Q = {}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16_split", "fp16_split", "bf16", "fp16"])
def test_32_qubit_chain_of_four_accuracy_matrix(prec):
    """2^32 outputs in every precision against the oracle on 10^5 sampled
    bins (seed 31), and against the FP64 GPU output over all bins."""
    m = cq()
    cm, E = syn.chain_instance(SEED_32Q, BONDS_32Q, NS_32Q)
    ents = [to_dev(e) for e in E]
    print(f"32q chain of four {prec}", flush=True)
    out = m.cq_reconstruct_fd(cm, ents, prec=prec)
    torch.cuda.synchronize()
    rng = np.random.default_rng(31)
    bins = rng.integers(0, 2 ** 32, size=100_000).astype(np.int64)
    got = out[torch.from_numpy(bins).to(DEV)].cpu().numpy().astype(np.float64)
    ref = rc.fd_per_bin(cm, E, bins)
    scale = rc.fd_per_bin(cm, [np.abs(e) for e in E], bins)
    err = np.abs(got - ref)
    rel = err / np.maximum(scale, 1e-300)
    line = (f"{prec}: sampled max abs {err.max():.3e}, TV estimate {2.0 ** 31 * err.mean():.3e}, "
            f"max err/scale {rel.max():.3e}, median err/scale {np.median(rel):.3e}")
    if prec == "fp64":
        _FP64_32Q["out"] = out
    elif "out" in _FP64_32Q:
        mx, tv = _full_vs(out, _FP64_32Q["out"])
        line += f"; vs FP64 GPU over 2^32: max abs {mx:.3e}, TV {tv:.3e}"
    print(line, flush=True)
    if prec == "fp64":
        assert err.max() < 1e-10
        assert np.all(err <= 1e-13 * scale + 1e-300)
    elif prec == "fp32":
        assert err.max() < 1e-6
        assert np.all(err <= 1e-5 * scale + fp32_floor(cm))
    elif prec == "bf16_split":
        assert err.max() < 1e-6
        assert np.all(err <= H16_REL[prec] * scale + fp32_floor(cm))
    elif prec == "fp16_split":
        # columns are scaled by powers of two before the FP16 conversion, so
        # hi + lo keeps 22 bits of every entry whatever its magnitude
        assert err.max() < 1e-6
        assert np.all(err <= 1e-5 * scale + fp32_floor(cm))
    else:
        assert np.all(err <= H16_REL[prec] * scale + fp32_floor(cm))
    if prec == "fp16":
        _FP64_32Q.clear()


# --- attribution: register-butterfly and general kernels ---------------------

def test_attribution_full_dd_shape_sampled_columns():
    """The DD subcircuit shape (22 slots: init slots 0, 1 for cuts 0, 1;
    measured slots 20, 21 for cuts 2, 3; 20 outputs), variants (16, 9, 2^22)
    uniform random on the device.  The oracle attributes a reduced subcircuit
    with the same cut slots and 8 outputs whose variant columns are gathered
    from 256 sampled output values b: its column s equals column b_s of the
    full result (the measured bits are the two least significant slots in
    both, so outcome(b, m) = 4 b + m)."""
    m = cq()
    sub = (22, [0, 1] + [-1] * 20, [-1] * 20 + [2, 3])
    gen = torch.Generator(device=DEV)
    gen.manual_seed(7)
    V = torch.rand((16, 9, 2 ** 22), dtype=torch.float64, device=DEV, generator=gen)
    print("attribution at the DD shape", flush=True)
    E = m.cq_attribute(sub, V)
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    bs = np.sort(rng.choice(2 ** 20, size=256, replace=False)).astype(np.int64)
    cols = (4 * bs[:, None] + np.arange(4)[None, :]).ravel()  # sample s, outcome m -> 4 s + m
    Vs = V[:, :, torch.from_numpy(cols).to(DEV)].cpu().numpy()
    small = (10, [0, 1] + [-1] * 8, [-1] * 8 + [2, 3])
    ref = at.attribute(small, Vs)
    got = E[:, torch.from_numpy(bs).to(DEV)].cpu().numpy()
    assert got.shape == ref.shape == (256, 256)
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("r,o", [(0, 0), (0, 2), (1, 1), (2, 2), (3, 1), (3, 2), (4, 1), (1, 3), (2, 4)])
def test_attribution_all_pass_shapes(r, o):
    """Random (non-physical) variant tensors through every attribution kernel
    shape: measured ends <= 2 and initialised ends <= 3 take the register
    butterflies, larger counts the general kernels.  Slots interleave init,
    output and measured roles, and cut ids are not in slot order."""
    rng = np.random.default_rng(100 + 10 * r + o)
    n = 3
    w = r + o + n
    roles = ["i"] * r + ["m"] * o + ["o"] * n
    rng.shuffle(roles)
    # an init slot may also be an output: make the first init slot one
    cuts = list(rng.permutation(r + o))
    init_cut, meas_cut = [-1] * w, [-1] * w
    ci = iter(cuts)
    for s, role in enumerate(roles):
        if role == "i":
            init_cut[s] = int(next(ci))
        elif role == "m":
            meas_cut[s] = int(next(ci))
    sub = (w, init_cut, meas_cut)
    V = rng.random((4 ** r, 3 ** o, 2 ** w))
    ref = at.attribute(sub, V)
    got = gpu_attribute(sub, V)
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("balance", [1, 0])
@pytest.mark.parametrize("prec", ["fp16_split", "fp16", "bf16_split"])
def test_32_qubit_chain_of_four_imbalanced_labels(prec, balance):
    """The accuracy matrix's per-label arm: the 32-qubit chain with label
    rows 2^+-20 apart inside each subcircuit (imbalance_labels: the exact
    result is unchanged), with and without the per-label balance, against the
    oracle on the same 10^5 sampled bins.  FP16-split with the balance must
    meet 1e-6; the BF16 forms do not depend on it (bit-identical either way)."""
    m = cq()
    cm, E = syn.chain_instance(SEED_32Q, BONDS_32Q, NS_32Q)
    Ei = imbalance_labels(cm, E)
    ents = [to_dev(e) for e in Ei]
    print(f"32q imbalanced labels {prec} balance {balance}", flush=True)
    try:
        m.cq_label_balance_enable(balance)
        out = m.cq_reconstruct_fd(cm, ents, prec=prec)
        torch.cuda.synchronize()
    finally:
        m.cq_label_balance_enable(1)
    rng = np.random.default_rng(31)
    bins = rng.integers(0, 2 ** 32, size=100_000).astype(np.int64)
    got = out[torch.from_numpy(bins).to(DEV)].cpu().numpy().astype(np.float64)
    del out
    ref = rc.fd_per_bin(cm, E, bins)
    scale = rc.fd_per_bin(cm, [np.abs(e) for e in E], bins)
    err = np.abs(got - ref)
    rel = err / np.maximum(scale, 1e-300)
    print(f"{prec} balance {balance}: sampled max abs {err.max():.3e}, TV estimate "
          f"{2.0 ** 31 * err.mean():.3e}, median err/scale {np.median(rel):.3e}", flush=True)
    if balance and prec == "fp16_split":
        assert err.max() < 1e-6
        assert np.all(err <= 1e-5 * scale + fp32_floor(cm))
    if prec == "bf16_split":
        assert err.max() < 1e-6
    if not balance and prec.startswith("fp16"):
        # without the balance the small label rows are lost in FP16
        assert np.median(rel) > 1e-3
