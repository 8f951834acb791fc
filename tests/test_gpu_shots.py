"""GPU parity of finite-shot emulation and the chi-square loss (Eq. 3)
against the oracle, through the C ABI.

Sampling takes every decision in integers (quantised probabilities, exact
prefix sums, Philox4x32-10 words, a 64 x 64 high product), so the device
frequencies must equal the oracle's bit for bit: on ragged widths that span
several blocks of 2048 entries (rows of one block, rows counted in LDS, rows
of more than 8192 blocks counted in global memory), on negative, zero,
unnormalised and single-spike rows, on seeds above 2^32, and at the
dynamic-definition subcircuit shape on sampled rows.  Tables with fewer
than 64 shots a block on average resolve light blocks in registers and list
the heavy ones; others resolve every block in LDS: both mixes are covered.
The loss is a floating-point sum in another order than the oracle's: it must
agree within 1e-12 of the sum of the terms' magnitudes, and repeat bit for
bit."""
import ctypes as C

import numpy as np
import pytest

from oracle import attribution as at
from oracle import reconstruct as rc
from oracle import shots
from oracle import statevector as sv
from workloads import circuits as wc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def cq():
    import paper_2205_05836_amd as m
    return m


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def gpu_freqs(P, n, seed):
    out = cq().cq_sample_shots(to_dev(P), n, seed)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _table(rng, rows, cols, kind):
    if kind == "dirichlet":
        return rng.dirichlet(np.full(cols, 0.5), size=rows)
    if kind == "uniform":     # unnormalised (row sums near 1.5), sampled in proportion
        return rng.random((rows, cols)) * (3.0 / cols)
    if kind == "mixed":       # quasi-probabilities: negatives, zero rows, entries above 1
        P = rng.normal(size=(rows, cols)) * 0.3
        P[0] = 0.0
        if rows > 2:
            P[2] = -np.abs(P[2])
        P[-1, cols // 2] = 1.7
        return P
    if kind == "spike":       # every shot of row 0 in one entry of a many-block row
        P = rng.dirichlet(np.ones(cols), size=rows)
        P[0] = 0.0
        P[0, (7 * cols) // 9] = 1.0
        return P
    raise ValueError(kind)


@pytest.mark.parametrize("rows,cols,n,seed,kind", [
    (1, 1, 1, 0, "uniform"),
    (1, 1, 1000, 5, "dirichlet"),
    (3, 37, 1000, 1, "dirichlet"),
    (4, 4095, 20000, 2, "uniform"),
    (5, 4097, 20000, 3, "dirichlet"),
    (2, 3 * 4096 + 5, 50000, 2 ** 40 + 17, "dirichlet"),
    (6, 300, 7777, 4, "mixed"),
    (16 * 9, 64, 1000, 9, "dirichlet"),
    (1, 1 << 20, 100000, 12345678901, "uniform"),
    (3, 10000, 100000, 6, "spike"),
    (4096, 16, 5000, 8, "dirichlet"),
    (1, (1 << 24) + 4099, 200000, 10, "dirichlet"),
    # fewer than 64 shots a block on average: light blocks resolve in
    # registers, heavy ones (the spike's block; Dirichlet blocks above 64)
    # are listed and resolved in LDS
    (2, 64 * 2048, 4000, 11, "spike"),
    (3, 100 * 2048 + 77, 6000, 13, "dirichlet"),
])
def test_frequencies_bit_exact(rows, cols, n, seed, kind):
    print(f"case rows={rows} cols={cols} shots={n} seed={seed} {kind}", flush=True)
    P = _table(np.random.default_rng(rows * 1000 + cols), rows, cols, kind)
    got = gpu_freqs(P, n, seed)
    want = shots.sample_frequencies(P, n, seed)
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    counts = np.rint(got * n)
    assert np.array_equal(counts / n, got)
    for r in range(rows):
        live = np.any(shots.quantise(P[r]) > 0)
        assert counts[r].sum() == (n if live else 0)


def test_variant_table_shape_and_repeat():
    """A (4^r, 3^o, 2^w) variant table keeps its shape; rows are the table's
    leading entries in row-major order; a repeat gives the same bits and a
    new seed other counts."""
    rng = np.random.default_rng(21)
    V = rng.dirichlet(np.ones(32), size=(4, 3)).reshape(4, 3, 32)
    P = to_dev(V)
    a = cq().cq_sample_shots(P, 4000, 77)
    b = cq().cq_sample_shots(P, 4000, 77)
    c = cq().cq_sample_shots(P, 4000, 78)
    torch.cuda.synchronize()
    assert a.shape == (4, 3, 32)
    assert torch.equal(a, b) and not torch.equal(a, c)
    assert np.array_equal(a.cpu().numpy(), shots.sample_frequencies(V, 4000, 77))


def test_full_dd_variant_shape_sampled_rows():
    """The dynamic-definition subcircuit's variant table: 16 x 9 rows of 2^22
    outcomes, 10^6 shots per row, uniform random entries generated on the
    device (rows summing to about 1).  Rows are independent streams (the row index is part of the
    counter), so the oracle checks sampled rows one at a time, bit for bit."""
    m = cq()
    rows, cols, n, seed = 16 * 9, 1 << 22, 1_000_000, 2022
    gen = torch.Generator(device=DEV)
    gen.manual_seed(5)
    P = torch.rand((rows, cols), dtype=torch.float64, device=DEV, generator=gen) * (2.0 / cols)
    print("shots at the DD variant shape", flush=True)
    F = m.cq_sample_shots(P, n, seed)
    torch.cuda.synchronize()
    sums = torch.round(F * n).sum(dim=1)
    assert torch.all(sums == n)
    for r in (0, 1, 77, rows - 1):
        want = shots.sample_counts(P[r].cpu().numpy(), n, seed, r) / float(n)
        assert np.array_equal(F[r].cpu().numpy(), want), r


def test_table_beyond_32_bit_indices():
    """Five rows of 2^29 + 7 outcomes (2.7e9 entries, offsets past 2^31):
    the last row, bit for bit against the oracle."""
    m = cq()
    rows, cols, n, seed = 5, (1 << 29) + 7, 100000, 77
    gen = torch.Generator(device=DEV)
    gen.manual_seed(9)
    P = torch.rand((rows, cols), dtype=torch.float64, device=DEV, generator=gen) * (2.0 / cols)
    print("shots past 2^31 entries", flush=True)
    F = m.cq_sample_shots(P, n, seed)
    torch.cuda.synchronize()
    assert torch.all(torch.round(F * n).sum(dim=1) == n)
    r = rows - 1
    want = shots.sample_counts(P[r].cpu().numpy(), n, seed, r) / float(n)
    got = F[r].cpu().numpy()
    del P, F
    assert np.array_equal(got, want)


def test_most_rows():
    """65535 rows (the largest count) of three outcomes."""
    rng = np.random.default_rng(65535)
    P = rng.dirichlet(np.ones(3), size=65535)
    got = gpu_freqs(P, 7, 3)
    want = shots.sample_frequencies(P, 7, 3)
    assert np.array_equal(got, want)


def test_sampling_arguments_rejected_before_launch():
    from paper_2205_05836_amd import _lib
    from paper_2205_05836_amd.api import _dev_ptr, _stream
    m = cq()
    P = to_dev(np.full((2, 8), 0.125))
    out = torch.full_like(P, -3.0)
    need = m.cq_sample_shots_workspace_size(2, 8, 100)
    ws = torch.empty(need - 8, dtype=torch.uint8, device=DEV)
    L = _lib.lib()
    st = L.cq_sample_shots(_dev_ptr(P), 2, 8, 100, C.c_uint64(1), _dev_ptr(out), _dev_ptr(ws),
                           C.c_size_t(need - 8), _stream(None))
    assert st == -5                                         # CQ_ERR_WORKSPACE
    for rows, cols, n, code in ((0, 8, 100, -1), (2, 0, 100, -1), (2, 8, 0, -1),
                                (70000, 8, 100, -2), (1, 1 << 35, 1, -2), (2, 8, 1 << 40, -2)):
        b = C.c_size_t()
        assert L.cq_sample_shots_workspace_size(rows, cols, n, C.byref(b)) == code
    torch.cuda.synchronize()
    assert torch.all(out == -3.0)
    with pytest.raises(m.CQError):
        m.cq_sample_shots(P, 0, 1)


@pytest.mark.parametrize("n,kind", [(1, "prob"), (7, "zeros"), (1000, "prob"), (4097, "quasi"),
                                    ((1 << 24) + 3, "prob"), ((1 << 26), "quasi")])
def test_chi2_matches_oracle(n, kind):
    print(f"chi2 n={n} {kind}", flush=True)
    rng = np.random.default_rng(n)
    if kind == "prob":
        a, b = rng.dirichlet(np.ones(n)), rng.dirichlet(np.ones(n))
    elif kind == "zeros":
        a = np.array([0.5, 0.0, 0.25, 0.0, 0.25, 0.0, 0.0])
        b = np.array([0.25, 0.0, 0.25, 0.5, 0.0, 0.0, 0.0])
    else:
        a = rng.normal(size=n) * 1e-3
        b = np.abs(rng.normal(size=n)) * 1e-3
        a[::5] = 0.0
        b[::5] = 0.0
    want = shots.chi2(a, b)
    s = a + b
    nz = s != 0
    mag = float(np.sum(np.abs((a[nz] - b[nz]) ** 2 / s[nz])))
    da, db = to_dev(a), to_dev(b)
    r1 = cq().cq_chi2(da, db)
    r2 = cq().cq_chi2(da, db)
    torch.cuda.synchronize()
    g1, g2 = float(r1.item()), float(r2.item())
    assert g1 == g2
    assert abs(g1 - want) <= 1e-12 * max(mag, 1e-300)
    if kind == "zeros":
        assert g1 == pytest.approx(0.25 ** 2 / 0.75 + 0.5 + 0.25, rel=1e-15)


def test_chi2_rejects_bad_arguments():
    from paper_2205_05836_amd import _lib
    from paper_2205_05836_amd.api import _dev_ptr, _stream
    L = _lib.lib()
    a = to_dev(np.ones(4))
    res = torch.full((1,), -1.0, dtype=torch.float64, device=DEV)
    ws = torch.empty(16, dtype=torch.uint8, device=DEV)
    assert L.cq_chi2(_dev_ptr(a), _dev_ptr(a), 4, _dev_ptr(res), _dev_ptr(ws), 16, _stream(None)) == -5
    assert L.cq_chi2(_dev_ptr(a), _dev_ptr(a), 0, _dev_ptr(res), _dev_ptr(ws), 16, _stream(None)) == -1
    torch.cuda.synchronize()
    assert float(res.item()) == -1.0


def test_finite_shot_cut_circuit_pipeline():
    """The 8-qubit one-cut circuit end to end on the device: sample each
    subcircuit's variant table, attribute, reconstruct (FP64), and the loss
    against the state vector; every step against the oracle's pipeline on
    the same seeds."""
    m = cq()
    cc = wc.two_way_circuit_8q(seed=0)
    subs = cc.subcircuits()
    Vs = [sv.variant_probabilities(s) for s in subs]
    truth = sv.probabilities(cc.n_qubits, cc.ops)
    for n in (1000, 100000):
        print(f"pipeline shots={n}", flush=True)
        Fo = [shots.sample_frequencies(V, n, seed=11 + c) for c, V in enumerate(Vs)]
        Eo = [at.attribute(s, F) for s, F in zip(subs, Fo)]
        po = rc.apply_out_perm(rc.fd_contract(subs, Eo), cc.out_perm())
        lo = shots.chi2(po, truth)
        Fg = [m.cq_sample_shots(to_dev(V), n, 11 + c) for c, V in enumerate(Vs)]
        for f, fo in zip(Fg, Fo):
            assert np.array_equal(f.cpu().numpy(), fo)
        Eg = [m.cq_attribute(s, f) for s, f in zip(subs, Fg)]
        pg = m.cq_reconstruct_fd(subs, Eg, prec="fp64", out_perm=cc.out_perm())
        lg = m.cq_chi2(pg.reshape(-1), to_dev(truth))
        torch.cuda.synchronize()
        assert np.max(np.abs(pg.cpu().numpy() - po)) < 1e-10
        s = po + truth
        nz = s != 0
        mag = float(np.sum(np.abs((po[nz] - truth[nz]) ** 2 / s[nz])))
        assert abs(float(lg.item()) - lo) <= 1e-9 * mag + 1e-15
