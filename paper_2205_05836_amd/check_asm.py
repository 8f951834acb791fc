"""Build-time check of the AMD assembly of the asynchronous, occupancy and
persistent label GEMMs (gemm.hip).

Those kernels move operand stages global -> LDS with global_load_lds_dwordx4
issued from inline asm and wait for them with hand-counted
`s_waitcnt vmcnt(N)`: vector memory operations of a wave retire in issue
order, so waiting until at most N are outstanding completes a stage only if
every later stage issued at least N of them.  Each such kernel states its
count per stage in an assembly comment (`; cq-vm-lpw LPW`, plus `out OUT`
for the persistent kernels, whose waits also count their output stores).
This check reads the assembly hipcc saved while compiling gemm.hip and
confirms, for every marked kernel:

* every basic block that issues DMA loads issues a multiple of LPW of them
  (stages are never split or partly dropped), and the kernel issues some;
* in the persistent kernels, each full output row is one store instruction
  of the expected width (16 bytes for FP32 output, 8 bytes per 16-bit
  plane), so a slab's store count is what the waits add up.

Extra vector memory instructions only make such waits longer, so they are
not an error.
"""
import re
import sys

_FUNC = re.compile(r"^(_Z\S+):")
_BLOCK = re.compile(r"^(\.LBB\d+_\d+:|; %bb\.\d+:)")
_MARK = re.compile(r";\s*cq-vm-lpw\s+(\d+)(?:\s+out\s+(\d+))?")


def _kernels(text):
    name, body = None, []
    for line in text.splitlines():
        m = _FUNC.match(line)
        if m:
            name, body = m.group(1), []
            continue
        if name is None:
            continue
        if line.startswith(".Lfunc_end"):
            yield name, body
            name = None
            continue
        body.append(line)


def check_text(text):
    """Problems found in assembly text (empty when it passes) and the number
    of marked kernels."""
    problems, marked = [], 0
    for name, body in _kernels(text):
        mark = None
        for line in body:
            m = _MARK.search(line)
            if m:
                mark = (int(m.group(1)), None if m.group(2) is None else int(m.group(2)))
                break
        if mark is None:
            continue
        marked += 1
        lpw, out = mark
        counts, cur, stores = [], 0, {}
        for line in body:
            if _BLOCK.match(line):
                counts.append(cur)
                cur = 0
                continue
            op = line.strip().split(" ", 1)[0]
            if op == "global_load_lds_dwordx4":
                cur += 1
            elif op.startswith("global_store") or op.startswith("buffer_store") or op.startswith("flat_store"):
                stores[op] = stores.get(op, 0) + 1
        counts.append(cur)
        issuing = [c for c in counts if c]
        if not issuing:
            problems.append(f"{name}: marked LPW {lpw} but issues no LDS-DMA loads")
        bad = [c for c in issuing if c % lpw]
        if bad:
            problems.append(f"{name}: basic blocks issue {bad} LDS-DMA loads, not multiples of LPW {lpw}")
        if out is not None:
            full = {0: "global_store_dwordx4", 1: "global_store_dwordx4", 2: "global_store_dwordx2"}[out]
            # ragged edges store element by element (uncounted, which only lengthens waits)
            allowed = {full, "global_store_dword", "global_store_short"}
            odd = sorted(op for op in stores if op not in allowed)
            if odd:
                problems.append(f"{name}: output stores {odd} besides one {full} per full row")
            if not stores.get(full):
                problems.append(f"{name}: no {full} for full output rows")
    return problems, marked


def check(path, min_marked=1):
    with open(path) as f:
        problems, marked = check_text(f.read())
    if marked < min_marked:
        problems.append(f"{path}: {marked} marked kernels, expected at least {min_marked}")
    return problems


if __name__ == "__main__":
    errs = check(sys.argv[1])
    for e in errs:
        print(e)
    sys.exit(1 if errs else 0)
