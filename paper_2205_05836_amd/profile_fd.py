"""Profiling driver: the 30-qubit full-definition workload (chain of three
10-output subcircuits, 4 + 4 cuts, seed 2) reconstructed once to warm up (the
GEMM autotuner picks its kernel variants then) and ``reps`` more times in one
precision, then one device-to-device copy of 1 GiB.

Inputs are generated on the host and copied in, so the only kernels that run
are the library's and the runtime's copy kernel; the copy moves a known
number of bytes and calibrates the HBM traffic counters (FETCH_SIZE,
WRITE_SIZE) read for the reconstruction kernels.

    python -m paper_2205_05836_amd.profile_fd bf16_split 3

Each counter (FETCH_SIZE, then WRITE_SIZE) is read in a run of its own under
``rocprofv3 --pmc``; ``summarize`` turns those runs' CSV files into the
per-launch HBM traffic of each GEMM step (calibrated by the copy):

    python -m paper_2205_05836_amd.profile_fd summarize OUT.json OUT.md BASE 3 bf16_split fp32 fp64

reads BASE/pmc_<prec>_<counter>/**/*counter_collection.csv.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

COPY_BYTES = 1 << 30


def main(argv):
    prec = argv[1] if len(argv) > 1 else "bf16_split"
    reps = int(argv[2]) if len(argv) > 2 else 3
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch

    import paper_2205_05836_amd as cq
    from workloads import synthetic as syn

    cm, E = syn.chain_instance(2, [4, 4], [10, 10, 10])
    ents = [torch.from_numpy(e).to("cuda:0") for e in E]
    dt = torch.float64 if prec == "fp64" else torch.float32
    out = torch.empty(2 ** 30, dtype=dt, device="cuda:0")
    torch.cuda.synchronize()
    # first call: the GEMM autotuner times its variants for these shapes
    cq.cq_reconstruct_fd(cm, ents, prec=prec, out=out)
    torch.cuda.synchronize()
    print("warm-up done", flush=True)
    for i in range(reps):
        cq.cq_reconstruct_fd(cm, ents, prec=prec, out=out)
        torch.cuda.synchronize()
        print(f"step {i} done", flush=True)
    del out
    a = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy of {COPY_BYTES} bytes done", flush=True)


SHORT = {"fp64": "gemm_f64", "fp32": "gemm_f32", "bf16": "gemm_bf16", "fp16": "gemm_f16",
         "bf16_split": "gemm_bf16x3", "fp16_split": "gemm_f16x3"}


def _dispatches(path):
    """[(dispatch id, kernel name, grid, counter value)] of one counter CSV,
    values summed over the rows of a dispatch, in dispatch order."""
    acc = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            d = int(r["Dispatch_Id"])
            v = float(r["Counter_Value"])
            if d in acc:
                acc[d][3] += v
            else:
                acc[d] = [d, r["Kernel_Name"], int(r["Grid_Size"]), v]
    return [tuple(acc[d]) for d in sorted(acc)]


def _csv_of(base, prec, counter):
    hits = glob.glob(os.path.join(base, f"pmc_{prec}_{counter}", "**", "*counter_collection.csv"),
                     recursive=True)
    if not hits:
        raise FileNotFoundError(f"no counter CSV for {prec} {counter} under {base}")
    return hits[0]


def summarize(argv):
    out_json, out_md, base, reps = argv[2], argv[3], argv[4], int(argv[5])
    precs = argv[6:]
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import paper_2205_05836_amd as cq
    from workloads import synthetic as syn

    cm = syn.chain_cutmap([4, 4], [10, 10, 10])
    sha = hashlib.sha256(open(os.path.join(root, "paper_2205_05836_amd", "csrc", "gemm.hip"),
                              "rb").read()).hexdigest()
    recs, md = [], ["# HBM traffic of the 30-qubit FD GEMMs (FETCH_SIZE, WRITE_SIZE)", "",
                    "Commands (repository root), one counter per run:", ""]
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        md.append(f"    rocprofv3 --kernel-include-regex \"gemm|prep|opy\" --pmc {c} --output-format csv "
                  f"-d gpurun_out/prof/pmc_<prec>_{c} -o run -- python3 -m "
                  f"paper_2205_05836_amd.profile_fd <prec> {reps}")
    md += ["", "Summary (this file and the JSON beside it):", "",
           f"    python3 -m paper_2205_05836_amd.profile_fd summarize {out_json} {out_md} "
           f"gpurun_out/prof {reps} {' '.join(precs)}", "",
           "The driver ends with a 1 GiB device-to-device copy (`__amd_rocclr_copyBuffer`, "
           "1 GiB read + 1 GiB written): its counters give the calibration factors "
           "(counter KiB x 1024 / true bytes).  Per GEMM step: the mean over the last "
           f"{reps} steps (the warm-up's autotuner runs excluded).", "",
           f"`gemm.hip` SHA-256 at the time: `{sha}`.", ""]
    for prec in precs:
        plan = cq.cq_plan_json(cm, prec)
        gsteps = [s for s in plan["steps"] if s["op"] == "gemm"]
        per = {}
        factor = {}
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            ds = _dispatches(_csv_of(base, prec, counter))
            copies = [d for d in ds if "copyBuffer" in d[1]]
            if not copies:
                raise RuntimeError(f"{prec} {counter}: no calibration copy in the trace")
            factor[counter] = copies[-1][3] * 1024.0 / COPY_BYTES
            gemms = [d for d in ds if "gemm" in d[1]][-reps * len(gsteps):]
            if len(gemms) != reps * len(gsteps):
                raise RuntimeError(f"{prec} {counter}: expected {reps * len(gsteps)} GEMM launches")
            for j, d in enumerate(gemms):
                per.setdefault(j % len(gsteps), {"name": d[1], "grid": d[2]}).setdefault(
                    counter, []).append(d[3])
        md += [f"## {prec}", "",
               f"Calibration: FETCH_SIZE factor {factor['FETCH_SIZE']:.4f}, "
               f"WRITE_SIZE factor {factor['WRITE_SIZE']:.4f}.", "",
               "| GEMM step | kernel | grid | FETCH_SIZE KiB (mean) | WRITE_SIZE KiB (mean) "
               "| HBM read GB | HBM write GB |",
               "|---|---|---:|---:|---:|---:|---:|"]
        for j, st in enumerate(gsteps):
            e = per[j]
            fk = sum(e["FETCH_SIZE"]) / len(e["FETCH_SIZE"])
            wk = sum(e["WRITE_SIZE"]) / len(e["WRITE_SIZE"])
            rd = fk * 1024.0 / factor["FETCH_SIZE"]
            wr = wk * 1024.0 / factor["WRITE_SIZE"]
            flops = 2.0 * st["Z"] * st["M"] * st["N"] * st["K"]
            recs.append({"precision": prec, "kernel": SHORT[prec], "kernel_name": e["name"],
                         "kernel_flops": flops, "grid": e["grid"], "fetch_kib": fk,
                         "write_kib": wk, "fetch_factor": factor["FETCH_SIZE"],
                         "write_factor": factor["WRITE_SIZE"],
                         "traffic_bytes_per_launch": int(round(rd + wr)),
                         "gemm_src_sha256": sha})
            short = e["name"].replace("void ", "").replace("(anonymous namespace)::", "")
            short = short[:short.index("(")] if "(" in short else short
            md.append(f"| {j} (Z {st['Z']}, {st['M']} x {st['N']} x {st['K']}) | `{short}` "
                      f"| {e['grid']} | {fk:.1f} | {wk:.1f} | {rd / 1e9:.4f} | {wr / 1e9:.4f} |")
        md.append("")
    with open(out_json, "w") as f:
        json.dump({"workload": "30-qubit FD, seed 2", "kernels": recs}, f, indent=1)
    with open(out_md, "w") as f:
        f.write("\n".join(md))


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "summarize":
        summarize(sys.argv)
    else:
        main(sys.argv)
