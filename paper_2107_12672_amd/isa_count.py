"""VALU instruction counts of the render kernels' inner loops, read from the
gfx950 assembly of the current source (a cross-check of the measured
counters).

    python -m paper_2107_12672_amd.isa_count [--write]

Compiles ``csrc/ddvr_kernels.hip`` with the library's flags to device
assembly and counts, for the absorption-only bf16 4-wave kernels, the VALU
instructions of one iteration of the forward's and of the closed-form
adjoint's cell-run loops (one run = the samples of a ray inside one cell).
It also counts, in ``csrc/ddvr_dfc.hip``, the VALU instructions of the
density-from-colour candidate loop (bf16 colour volume): one candidate.
``--write`` stores the counts with the source hashes in
``profiles/valu_per_run_c3.json`` and ``profiles/valu_per_candidate_dfc.json``,
the second of which the benchmark reads (the first documents the cell-run loops).
"""
from __future__ import annotations

import hashlib
import json
import os
import re
import subprocess
import sys
import tempfile

from . import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(ROOT, "profiles", "valu_per_run_c3.json")
OUT_DFC = os.path.join(ROOT, "profiles", "valu_per_candidate_dfc.json")
DFC_SOURCES = ["paper_2107_12672_amd/csrc/ddvr_dfc.hip", "paper_2107_12672_amd/csrc/ddvr_internal.h"]
DFC = "_ZN4ddvr12_GLOBAL__N_120k_density_from_colorILi2EEEvNS_9DfcParamsE"
KERNEL_SOURCES = ["paper_2107_12672_amd/csrc/ddvr_kernels.hip",
                  "paper_2107_12672_amd/csrc/ddvr_internal.h"]
FWD = "_ZN4ddvr8k_renderILi0ELi2ELi4ELi0ELb0EEEvNS_12LaunchParamsE"
FUSED = "_ZN4ddvr8k_renderILi0ELi2ELi4ELi2ELb0EEEvNS_12LaunchParamsE"


def strip_comments(text: str) -> str:
    """C++ source without its comments, whitespace runs collapsed to one space
    (string and character literals kept as written)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash(sources=None) -> str:
    """Hash of the code of the kernel sources (comments and layout ignored):
    the key under which measured counters and counts of these kernels are
    stored, so that they stay valid across comment edits and go stale with
    any change to the code."""
    h = hashlib.sha256()
    for rel in (sources or KERNEL_SOURCES):
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(strip_comments(f.read()).encode())
    return h.hexdigest()[:16]


def assembly(src: str = "ddvr_kernels.hip") -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in _build.HIPCC_FLAGS if f != "-fPIC"]
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "k.s")
        subprocess.check_call([hipcc] + flags + ["--cuda-device-only", "-S", "-o", out,
                                                 os.path.join(_build.CSRC, src)],
                              stderr=subprocess.DEVNULL)
        with open(out) as f:
            return f.read()


def _kernel(asm: str, sym: str):
    lines = asm.split("\n")
    start = next(i for i, l in enumerate(lines) if l.startswith(sym + ":"))
    end = next(i for i in range(start, len(lines)) if lines[i].startswith(".Lfunc_end"))
    return lines[start:end]


def _loops(lines):
    """Innermost loops: {header: [(block header line, [mnemonics]), ...]},
    from the compiler's loop annotations on block labels ("in Loop:
    Header=BBx" on member blocks, "This Inner Loop Header" on the header)."""
    loops, cur, members = {}, None, None
    for i, l in enumerate(lines):
        is_label = re.match(r"^(\.LBB\S+):", l) or l.startswith("; %bb.")
        if is_label:
            cur = None
            m = re.match(r"^\.L(BB\S+):", l)
            nxt = lines[i + 1] if i + 1 < len(lines) else ""
            if m and ("Inner Loop Header" in l or "Inner Loop Header" in nxt):
                cur = m.group(1)
            else:
                h = re.search(r"in Loop: Header=(BB\S+)", l)
                if h:
                    cur = h.group(1)
            if cur is not None:
                members = []
                loops.setdefault(cur, []).append((l, members))
            continue
        t = l.strip()
        if cur is not None and l.startswith("\t") and t and not t.startswith((".", ";")):
            members.append(t.split()[0])
    return loops


def _inner(lines):
    """Innermost loops only: headers whose own label carries the inner-loop mark."""
    marked = set()
    for i, l in enumerate(lines):
        m = re.match(r"^\.L(BB\S+):", l)
        if m and ("Inner Loop Header" in l or
                  (i + 1 < len(lines) and "Inner Loop Header" in lines[i + 1])):
            marked.add(m.group(1))
    return {h: b for h, b in _loops(lines).items() if h in marked}


def count(asm: str) -> dict:
    """Absorption-only bf16 kernels: the forward marches one cell run per
    iteration (the innermost loop with the four ds_read2_b32 of a cell's
    corners from the brick), the fused kernel's closed-form adjoint one run per
    iteration (the innermost loop that adds 8 corner sums to the brick,
    ds_add_u32, and finds the run's end with ceil/floor, without an
    exponential: the inversion loops have one)."""
    fwd = adj = None
    for blocks in _inner(_kernel(asm, FWD)).values():
        ins = [x for _, blk in blocks for x in blk]
        if ins.count("ds_read2_b32") == 4:
            fwd = sum(1 for x in ins if x.startswith("v_"))
            break
    for blocks in _inner(_kernel(asm, FUSED)).values():
        ins = [x for _, blk in blocks for x in blk]
        if ins.count("ds_add_u32") != 8 or any(x.startswith("v_exp_f32") for x in ins):
            continue
        if not any(x.startswith(("v_ceil_f32", "v_floor_f32")) for x in ins):
            continue
        adj = sum(1 for x in ins if x.startswith("v_"))
        break
    if fwd is None or adj is None:
        raise RuntimeError("run loops not found in the assembly")
    return {"forward_valu_per_run": fwd, "adjoint_valu_per_run": adj}


def count_dfc(asm: str) -> dict:
    """VALU instructions of the candidate loop (the innermost loop holding the
    log of the extinction term)."""
    for blocks in _inner(_kernel(asm, DFC)).values():
        ins = [x for _, blk in blocks for x in blk]
        if any(x.startswith("v_log_f32") for x in ins):
            return {"valu_per_candidate": sum(1 for x in ins if x.startswith("v_"))}
    raise RuntimeError("candidate loop not found in the assembly")


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    res = count(assembly())
    res["kernel_source_sha"] = source_hash()
    res["kernels"] = {"forward": FWD, "fused": FUSED}
    dfc = count_dfc(assembly("ddvr_dfc.hip"))
    dfc["kernel_source_sha"] = source_hash(DFC_SOURCES)
    dfc["kernel"] = DFC
    print(json.dumps(res, indent=1))
    print(json.dumps(dfc, indent=1))
    if "--write" in argv:
        os.makedirs(os.path.dirname(OUT), exist_ok=True)
        with open(OUT, "w") as f:
            json.dump(res, f, indent=1)
        with open(OUT_DFC, "w") as f:
            json.dump(dfc, f, indent=1)


if __name__ == "__main__":
    main()
