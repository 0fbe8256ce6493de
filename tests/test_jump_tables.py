"""Static check of the computed jumps in the built device code.

The wide elimination step enters one of 16 same-length instruction variants
(one per broadcast lane of the pivot row) through s_getpc / s_setpc.  A wrong
case length or base offset would send a wavefront into the middle of an
instruction, so every table in the built code objects is checked here: for
each p in [0, 16) the jump target must start the variant of p, every
broadcast in that variant must read lane p, the variants must be the same
instructions apart from that lane, each must have the stated byte length, and
all must branch to the common end right after the last one.  Runs on the CPU against the objects of the last build.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_2608_01332_amd", "_build")
LLVM = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"


def _tools():
    need = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-objdump")]
    return need if all(os.path.exists(t) for t in need) else None


def _disassemble(obj: str, tmp) -> list:
    objcopy, bundler, objdump = _tools()
    fat = os.path.join(tmp, "fatbin")
    co = os.path.join(tmp, "device.co")
    subprocess.run([objcopy, f"--dump-section=.hip_fatbin={fat}", obj, os.path.join(tmp, "host.o")],
                   check=True, capture_output=True)
    subprocess.run([bundler, "--type=o", f"--targets={TARGET}", f"--input={fat}", f"--output={co}", "--unbundle"],
                   check=True, capture_output=True)
    out = subprocess.run([objdump, "-d", "--mcpu=gfx950", co], check=True, capture_output=True, text=True).stdout
    ins = []
    for line in out.split("\n"):
        m = re.match(r"\s+(\S.*?)\s*//\s+([0-9A-F]+):", line)
        if m:
            ins.append((int(m.group(2), 16), m.group(1)))
    return ins


def check_tables(ins: list) -> tuple:
    """Number of jump tables found and the list of problems."""
    at = {a: i for i, (a, _) in enumerate(ins)}
    problems, n = [], 0
    for i, (_, text) in enumerate(ins):
        if not text.startswith("s_getpc_b64 s[40:41]"):
            continue
        n += 1
        head = [t for _, t in ins[i + 1:i + 7]]
        if not (head[0].startswith("s_and_b32 s42,") and head[0].endswith(", 15")):
            problems.append(f"table {n}: no lane mask: {head[0]}")
            continue
        mul = re.fullmatch(r"s_mul_i32 s42, s42, (0x[0-9a-f]+|\d+)", head[1])
        add = re.fullmatch(r"s_add_u32 s42, s42, (0x[0-9a-f]+|\d+)", head[2])
        if not (mul and add and head[3] == "s_add_u32 s40, s40, s42" and head[4] == "s_addc_u32 s41, s41, 0"
                and head[5] == "s_setpc_b64 s[40:41]"):
            problems.append(f"table {n}: unexpected head {head}")
            continue
        base = ins[i + 1][0] + int(add.group(1), 0)  # s_getpc_b64 yields the next instruction's address
        case = int(mul.group(1), 0)
        end = base + 16 * case
        for p in range(16):
            tgt = base + p * case
            if tgt not in at:
                problems.append(f"table {n}, p {p}: no instruction starts at {tgt:#x}")
                continue
            k = at[tgt]
            body = []
            while k < len(ins) and not ins[k][1].startswith("s_branch"):
                text_k = ins[k][1]
                if "row_newbcast" in text_k and re.search(rf"row_newbcast:{p}(\s|$)", text_k) is None:
                    problems.append(f"table {n}, p {p}: {text_k}")
                body.append(re.sub(r"row_newbcast:\d+", "row_newbcast:P", text_k))
                k += 1
            if not any("row_newbcast:P" in t for t in body):
                problems.append(f"table {n}, p {p}: no broadcast of the pivot row")
            if p == 0:
                first = body
            elif body != first:
                problems.append(f"table {n}, p {p}: the variant differs from the variant of p = 0")
            if k == len(ins):
                problems.append(f"table {n}, p {p}: no branch to the end")
                continue
            if ins[k][0] + 4 - tgt != case:
                problems.append(f"table {n}, p {p}: variant of {ins[k][0] + 4 - tgt} bytes, not {case}")
            dest = ins[k][0] + 4 + 4 * int(ins[k][1].split()[1])
            if dest != end:
                problems.append(f"table {n}, p {p}: branches to {dest:#x}, not {end:#x}")
        if end not in at or not ins[at[end]][1].startswith("s_nop"):
            problems.append(f"table {n}: the end {end:#x} does not open with the wait states")
    return n, problems


@pytest.mark.parametrize("src,nb", [("inst12", 12), ("inst16", 16)])
def test_dpp_jump_tables(src, nb, tmp_path):
    obj = os.path.join(BUILD, f"{src}.hip.o")
    if _tools() is None or not os.path.exists(obj):
        pytest.skip("needs the ROCm LLVM tools and a build of the solver library")
    n, problems = check_tables(_disassemble(obj, str(tmp_path)))
    assert n > 0, "no jump table found in the wide-layout code"
    assert not problems, "\n".join(problems[:20])


def _synthetic(fmas: int, stated: int) -> list:
    """A table as the compiler lays it out, with `fmas` FMAs per variant and a
    stated variant length of `stated` bytes."""
    ins, a = [], 0x1000

    def emit(t, size):
        nonlocal a
        ins.append((a, t))
        a += size

    emit("s_getpc_b64 s[40:41]", 4)
    emit("s_and_b32 s42, s10, 15", 4)
    emit(f"s_mul_i32 s42, s42, {stated:#x}", 8)
    emit("s_add_u32 s42, s42, 32", 8)
    emit("s_add_u32 s40, s40, s42", 4)
    emit("s_addc_u32 s41, s41, 0", 4)
    emit("s_setpc_b64 s[40:41]", 4)
    end = a + 16 * (8 * fmas + 4)
    for p in range(16):
        for _ in range(fmas):
            emit(f"v_fmac_f64_dpp v[0:1], v[0:1], v[2:3] row_newbcast:{p} row_mask:0xf bank_mask:0xf", 8)
        emit(f"s_branch {(end - a - 4) // 4}", 4)
    emit("s_nop 1", 4)
    return ins


def test_checker_accepts_a_well_formed_table():
    assert check_tables(_synthetic(2, 20)) == (1, [])


def test_checker_catches_a_wrong_case_length():
    n, problems = check_tables(_synthetic(3, 20))
    assert n == 1 and any("bytes, not 20" in t for t in problems)
