"""cq_reconstruct_fd_noalloc (full definition on the library's fixed scratch
array, for callers that cannot allocate) against cq_reconstruct_fd with a
caller workspace, through the C ABI.  Both run the same kernels on the same
plan, so the outputs must agree bit for bit.  Two calls in a row, the second
smaller, show that the scratch left by one call does not leak into the next;
a reconstruction whose workspace exceeds the scratch is rejected before any
launch and leaves the output untouched."""
import numpy as np
import pytest

from workloads import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def cq():
    import paper_2205_05836_amd as m
    return m


def entries(seed, bonds, ns):
    cm, E = syn.chain_instance(seed, bonds, ns)
    return cm, [torch.from_numpy(e).to(DEV) for e in E]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16_split", "fp16_split", "bf16"])
def test_noalloc_matches_workspace_path_twice(prec):
    m = cq()
    dt = torch.float64 if prec == "fp64" else torch.float32
    # a 24-qubit chain (tens of MiB of scratch), then a 15-qubit one with a
    # permuted output order
    cases = [(41, [3, 3], [8, 8, 8], None),
             (42, [2, 1], [5, 4, 6], [int(x) for x in np.random.default_rng(4).permutation(15)])]
    for seed, bonds, ns, perm in cases:
        cm, ents = entries(seed, bonds, ns)
        need = m.cq_fd_workspace_size(cm, prec, perm)
        assert 0 < need <= (64 << 20)
        n = sum(ns)
        print(f"noalloc {prec} chain {ns} bonds {bonds}: {need} bytes of scratch", flush=True)
        ref = m.cq_reconstruct_fd(cm, ents, prec=prec, out_perm=perm)
        out = torch.full((2 ** n,), float("nan"), dtype=dt, device=DEV)
        m.cq_reconstruct_fd_noalloc(cm, ents, out, prec=prec, out_perm=perm)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (prec, ns)


def test_noalloc_rejects_oversized_before_launch():
    m = cq()
    cm = syn.chain_cutmap([4, 4], [10, 10, 10])
    assert m.cq_fd_workspace_size(cm, "fp32") > (64 << 20)
    ents = [torch.zeros(4 ** k, 2 ** 10, dtype=torch.float64, device=DEV)
            for k in syn.chain_ks([4, 4], 3)]
    out = torch.full((2 ** 30,), -1.0, dtype=torch.float32, device=DEV)
    with pytest.raises(m.CQError) as ei:
        m.cq_reconstruct_fd_noalloc(cm, ents, out, prec="fp32")
    assert "CQ_ERR_WORKSPACE" in str(ei.value)
    torch.cuda.synchronize()
    assert bool(torch.all(out == -1.0))
