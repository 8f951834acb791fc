"""Tuned GEMM choices kept across processes (cq_autotune_save / _load and
CQ_TUNE_CACHE): a process that tunes writes the file, a fresh process that
reads it and captures its first reconstruction into a graph launches the
tuned variants (no timing happens under capture) and gets the eager result
bit for bit."""
import json
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_CHILD = r'''
import json, sys
sys.path.insert(0, sys.argv[1])
import torch
import paper_2205_05836_amd as cq
from workloads import synthetic as syn
mode = sys.argv[2]
cm, E = syn.chain_instance(31, [2, 2], [8, 8, 8])
ents = [torch.from_numpy(e).to("cuda:0") for e in E]
n = 24
ws = torch.empty(max(cq.cq_fd_workspace_size(cm, "bf16_split"), 1), dtype=torch.uint8, device="cuda:0")
out = torch.empty(2 ** n, dtype=torch.float32, device="cuda:0")
if mode == "tune":
    cq.cq_reconstruct_fd(cm, ents, prec="bf16_split", out=out, workspace=ws)
    torch.cuda.synchronize()
else:
    # first launch under capture: only choices loaded from the file can apply
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        cq.cq_reconstruct_fd(cm, ents, prec="bf16_split", out=out, workspace=ws,
                             stream=torch.cuda.current_stream())
    g.replay()
    torch.cuda.synchronize()
    captured = out.clone()
    eager = torch.empty_like(out)
    cq.cq_reconstruct_fd(cm, ents, prec="bf16_split", out=eager, workspace=ws)
    torch.cuda.synchronize()
    print("EQUAL", bool(torch.equal(captured, eager)))
print("JSON", json.dumps(cq.cq_autotune_json()))
'''


def _run(mode, cache, tmp_path):
    script = tmp_path / "child.py"
    script.write_text(_CHILD)
    env = dict(os.environ, CQ_TUNE_CACHE=str(cache), CQ_AUTOTUNE="1")
    print(f"autotune child {mode}", flush=True)
    r = subprocess.run([sys.executable, str(script), ROOT, mode], capture_output=True, text=True,
                       timeout=240, env=env)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    lines = {l.split(" ", 1)[0]: l.split(" ", 1)[1] for l in r.stdout.splitlines() if " " in l}
    return lines


def test_tuning_file_carries_choices_into_a_capturing_process(tmp_path):
    cache = tmp_path / "tune.txt"
    first = _run("tune", cache, tmp_path)
    tuned = json.loads(first["JSON"])
    assert tuned, "the tuning process timed no shape"
    text = cache.read_text()
    assert text.count("cq-tune-1 ") == len(tuned)
    second = _run("capture", cache, tmp_path)
    assert second["EQUAL"] == "True"
    loaded = {(e["prec"], e["M"], e["N"], e["K"], e["Z"]): (e["variant"], e["ms"])
              for e in json.loads(second["JSON"])}
    for e in tuned:
        # the same choice and the first process's timings: nothing was re-timed
        assert loaded[(e["prec"], e["M"], e["N"], e["K"], e["Z"])] == (e["variant"], e["ms"])
