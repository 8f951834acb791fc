"""The build-time assembly check of the asynchronous and persistent label
GEMMs (paper_2205_05836_amd/check_asm.py): the assembly of the current build
passes it, and the check catches a stage that lost one LDS-DMA load and a
persistent kernel whose full output rows are stored by narrower
instructions.  No GPU."""
import os

import pytest

from paper_2205_05836_amd import build, check_asm

ASM = build._device_asm("gemm.hip")


@pytest.fixture(scope="module")
def text():
    if not os.path.exists(ASM):
        pytest.skip("no saved device assembly (run the build first)")
    with open(ASM) as f:
        return f.read()


def test_built_assembly_passes(text):
    problems, marked = check_asm.check_text(text)
    assert problems == []
    # every asynchronous, occupancy and persistent 16-bit / FP32 kernel is marked
    assert marked >= 40


def test_a_missing_dma_load_is_caught(text):
    i = text.index("global_load_lds_dwordx4")
    bad = text[:i] + "v_nop" + text[i + len("global_load_lds_dwordx4"):]
    problems, _ = check_asm.check_text(bad)
    assert problems and "not multiples of LPW" in problems[0]


def test_a_split_row_store_is_caught(text):
    # the first persistent kernel with FP32 output: its first 16-byte row store becomes 8 bytes
    start = text.index("cq-vm-lpw 4 out 1")
    i = text.index("global_store_dwordx4", start)
    bad = text[:i] + "global_store_dwordx2" + text[i + len("global_store_dwordx4"):]
    problems, _ = check_asm.check_text(bad)
    assert any("output stores" in p for p in problems)
