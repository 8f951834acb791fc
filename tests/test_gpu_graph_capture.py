"""Entry points captured into a HIP graph by the caller (torch.cuda.graph):
finite-shot sampling with the chi-square loss, attribution with the full
definition, and the state vector.  None of them allocates, synchronises or
clears memory with a memset, so each can be captured; every replay must
reproduce the eager result bit for bit, with eager work on the same buffers'
neighbours and synchronisations between the replays."""
import numpy as np
import pytest

from oracle import statevector as sv
from workloads import circuits as wc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def cq():
    import paper_2205_05836_amd as m
    return m


def _replays(g, outputs, eager, noise):
    for r in range(3):
        noise(r)
        torch.cuda.synchronize()
        for o in outputs:
            o.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outputs, eager):
            assert torch.equal(o, e), r


def test_shots_and_chi2_captured():
    m = cq()
    rows, cols, n = 144, 1 << 16, 20000
    gen = torch.Generator(device=DEV)
    gen.manual_seed(3)
    P = torch.rand((rows, cols), dtype=torch.float64, device=DEV, generator=gen) * (2.0 / cols)
    F = torch.empty_like(P)
    ws = torch.empty(m.cq_sample_shots_workspace_size(rows, cols, n), dtype=torch.uint8, device=DEV)
    cws = torch.empty(m.cq_chi2_workspace_size(), dtype=torch.uint8, device=DEV)
    res = torch.empty(1, dtype=torch.float64, device=DEV)
    m.cq_sample_shots(P, n, 5, out=F, workspace=ws)
    m.cq_chi2(F.reshape(-1), P.reshape(-1), out=res, workspace=cws)
    torch.cuda.synchronize()
    eager = [F.clone(), res.clone()]
    print("capture shots + chi2", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        m.cq_sample_shots(P, n, 5, out=F, workspace=ws)
        m.cq_chi2(F.reshape(-1), P.reshape(-1), out=res, workspace=cws)
    F2 = torch.empty_like(P)

    def noise(r):   # eager calls between replays reuse the workspace with other seeds
        m.cq_sample_shots(P, n, 100 + r, out=F2, workspace=ws)
        m.cq_chi2(F2.reshape(-1), P.reshape(-1), out=torch.empty_like(res), workspace=cws)

    _replays(g, [F, res], eager, noise)


def test_attribution_and_fd_captured():
    m = cq()
    cc = wc.two_way_circuit_20q(1)
    subs = cc.subcircuits()
    V = [torch.from_numpy(sv.variant_probabilities(s)).to(DEV) for s in subs]
    E = [m.cq_attribute(s, v) for s, v in zip(subs, V)]
    aws = [torch.empty(max(m.cq_attribute_workspace_size(s), 1), dtype=torch.uint8, device=DEV)
           for s in subs]
    fws = torch.empty(max(m.cq_fd_workspace_size(subs, "fp32", cc.out_perm()), 1), dtype=torch.uint8,
                      device=DEV)
    out = torch.empty(2 ** 20, dtype=torch.float32, device=DEV)
    for s, v, e, w in zip(subs, V, E, aws):
        m.cq_attribute(s, v, entries=e, workspace=w)
    m.cq_reconstruct_fd(subs, E, prec="fp32", out_perm=cc.out_perm(), out=out, workspace=fws)
    torch.cuda.synchronize()
    eager = [out.clone()] + [e.clone() for e in E]
    print("capture attribution + fd", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for s, v, e, w in zip(subs, V, E, aws):
            m.cq_attribute(s, v, entries=e, workspace=w)
        m.cq_reconstruct_fd(subs, E, prec="fp32", out_perm=cc.out_perm(), out=out, workspace=fws)

    def noise(r):
        m.cq_reconstruct_fd(subs, E, prec="fp64", out_perm=cc.out_perm())

    _replays(g, [out] + E, eager, noise)
    ref = sv.probabilities(cc.n_qubits, cc.ops)
    assert np.max(np.abs(out.cpu().numpy().astype(np.float64) - ref)) < 1e-6


def test_state_vector_captured():
    m = cq()
    rng = np.random.default_rng(4)
    ops = [wc.Op("u", (int(rng.integers(16)),), wc.haar_u2(rng)) if rng.random() < 0.6 else
           wc.Op("cz", tuple(int(x) for x in rng.choice(16, size=2, replace=False))) for _ in range(120)]
    ws = torch.empty(m.cq_simulate_workspace_size(16), dtype=torch.uint8, device=DEV)
    out = torch.empty(2 ** 16, dtype=torch.float64, device=DEV)
    m.cq_simulate_probabilities(16, ops, out=out, workspace=ws)
    torch.cuda.synchronize()
    eager = [out.clone()]
    print("capture state vector", flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        m.cq_simulate_probabilities(16, ops, out=out, workspace=ws)

    def noise(r):
        m.cq_simulate_probabilities(16, ops[: 10 * (r + 1)], out=torch.empty_like(out), workspace=ws)

    _replays(g, [out], eager, noise)
    assert np.max(np.abs(out.cpu().numpy() - sv.probabilities(16, ops))) < 1e-12
