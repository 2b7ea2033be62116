"""Instruction counts of the built marcher's sample loops, read from the
library's own gfx950 code object (the code that runs).

The batched compositing kernel's cost per sample is the number of vector-ALU
instructions its inner loop issues per sample: the benchmark multiplies that
by the composited samples of a launch to get the VALU work the samples
required, the numerator of the instruction-issue roofline.

The code object is taken from the ``.hip_fatbin`` section of ``librtvol.so``
(offload bundles, one per source file), unbundled for gfx950 and
disassembled with the ROCm LLVM tools; only the named kernel is
disassembled.  The loop is found structurally: a backward-branch range with
no workgroup barrier whose body holds, per sample, one volume load and the
transfer-function reads of one compositing step (either the two table
entries as two 16-byte LDS reads, or, where colour is composited under the
wave's vote, the two opacities as one paired 4-byte read and the two colours
as two 12-byte reads), and, among
such loops of the kernel, the one with the fewest VALU instructions per
sample (the plain compositing loop; thresholding adds its window test).

A sample whose interpolated opacity is zero in every lane of the wavefront
skips its colour block: a branch on the wave's vote.  The instructions such
branches jump over are counted apart, so the profile gives the cost of a
sample that composites and of one that the whole wave finds transparent; the
cost of a launch lies between the two and is measured by the hardware
counters, not here.
"""
from __future__ import annotations

import os
import re
import subprocess
import tempfile
from typing import Dict, List, Optional, Tuple

LLVM_BIN = "/opt/rocm/llvm/bin"
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"
_INS = re.compile(r"^\s+([a-z_0-9]+)(.*?)//\s*([0-9A-F]+):")
_TGT = re.compile(r"<([^>+]+)\+0x([0-9a-f]+)>")


def _tool(name: str) -> str:
    p = os.path.join(LLVM_BIN, name)
    return p if os.path.exists(p) else name


def _code_objects(lib_path: str, workdir: str) -> List[str]:
    """gfx950 code objects of every offload bundle in the library."""
    fat = os.path.join(workdir, "fatbin.bin")
    subprocess.run([_tool("llvm-objcopy"), f"--dump-section=.hip_fatbin={fat}", lib_path, os.devnull],
                   check=True, capture_output=True)
    data = open(fat, "rb").read()
    starts = [m.start() for m in re.finditer(re.escape(MAGIC), data)]
    out = []
    for k, s in enumerate(starts):
        e = starts[k + 1] if k + 1 < len(starts) else len(data)
        b = os.path.join(workdir, f"bundle{k}.bin")
        open(b, "wb").write(data[s:e])
        co = os.path.join(workdir, f"bundle{k}.co")
        r = subprocess.run([_tool("clang-offload-bundler"), "--unbundle", "--type=o", f"--input={b}",
                            f"--targets={TARGET}", f"--output={co}"], capture_output=True)
        if r.returncode == 0 and os.path.getsize(co) > 0:
            out.append(co)
    return out


def _symbols(co: str) -> List[str]:
    r = subprocess.run([_tool("llvm-readelf"), "--symbols", "--wide", co], check=True, capture_output=True,
                       text=True)
    return [ln.split()[-1] for ln in r.stdout.splitlines() if " FUNC " in ln]


def _disassemble(co: str, sym: str) -> List[Tuple[int, str, str]]:
    r = subprocess.run([_tool("llvm-objdump"), "-d", "--mcpu=gfx950", f"--disassemble-symbols={sym}", co],
                       check=True, capture_output=True, text=True)
    base = None
    ins = []
    for ln in r.stdout.splitlines():
        m = re.match(r"^([0-9a-f]+) <(.+)>:", ln)
        if m:
            base = int(m.group(1), 16)
            continue
        m = _INS.match(ln)
        if m and base is not None:
            ins.append((int(m.group(3), 16), m.group(1), ln))
    return ins


def _loops(ins: List[Tuple[int, str, str]]) -> List[Tuple[int, int]]:
    """(first, last) instruction indices of the sample loops: ranges of
    backward branches that hold no workgroup barrier (the outer loop over
    claimed blocks has one), keeping the widest of nested ranges (a loop
    unrolled by two has a second backward branch, its mid-body exit, inside
    its own range)."""
    addr_idx = {a: k for k, (a, _, _) in enumerate(ins)}
    base = ins[0][0] if ins else 0
    back = []
    for k, (a, op, ln) in enumerate(ins):
        if not op.startswith("s_branch") and not op.startswith("s_cbranch"):
            continue
        m = _TGT.search(ln)
        if not m:
            continue
        t = base + int(m.group(2), 16)
        if t <= a and t in addr_idx:
            lo = addr_idx[t]
            if not any(op2 == "s_barrier" for _, op2, _ in ins[lo:k + 1]):
                back.append((lo, k))
    outer = [r for r in back if not any(o != r and o[0] <= r[0] and r[1] <= o[1] for o in back)]
    return sorted(set(outer))


def loop_profile(lib_path: str, kind: int, layout: int, kernel: str = "march_batch_kernel",
                 tail: Optional[str] = None) -> Optional[Dict]:
    """VALU (and other) instructions per sample of the compositing loop of
    kernel<kind, layout, ...> in the built library, or None when not found:
    `valu_per_sample` for a sample that composites, and
    `valu_per_transparent_sample` for one whose wave skips the colour block.
    `tail` is the mangled rest of the template arguments (the batched kernel
    has none; the single-view kernel's fixed-step compositing instantiation,
    <kind, layout, false, true>, is the default for it)."""
    if tail is None:
        tail = "Lb0ELb1E" if kernel == "march_plain_kernel" else ""
    with tempfile.TemporaryDirectory() as wd:
        for co in _code_objects(lib_path, wd):
            pat = re.compile(r"\d+" + kernel + rf"ILi{kind}ELi{layout}E{tail}E")
            syms = [s for s in _symbols(co) if pat.search(s)]
            if not syms:
                continue
            ins = _disassemble(co, syms[0])
            best = None
            addr_idx = {a: k for k, (a, _, _) in enumerate(ins)}
            base = ins[0][0] if ins else 0
            for lo, hi in _loops(ins):
                body = [op for _, op, _ in ins[lo:hi + 1]]
                loads = sum(op.startswith(("buffer_load", "global_load")) for op in body)
                voted = body.count("ds_read2_b32")
                if voted >= 1 and body.count("ds_read_b96") == 2 * voted:
                    samples = voted   # opacities apart, colours under the wave's vote
                else:
                    wide = body.count("ds_read_b128")
                    samples = wide // 2 if wide % 2 == 0 else 0   # both table entries whole
                if samples < 1 or loads != samples:
                    continue
                valu = sum(op.startswith("v_") for op in body)
                skipped = set()
                after_alpha = False   # the wave's vote follows the sample's opacity read
                for k in range(lo, hi + 1):
                    a, op, ln = ins[k]
                    if op == "ds_read2_b32":
                        after_alpha = True
                    elif op.startswith(("buffer_load", "global_load")):
                        after_alpha = False
                    m = _TGT.search(ln)
                    if not op.startswith("s_cbranch_vcc") or not m or not after_alpha:
                        continue
                    after_alpha = False
                    t = addr_idx.get(base + int(m.group(2), 16))
                    if t is None:
                        continue
                    # a forward branch inside the body skips up to its target; one
                    # back to the loop head skips the rest of the body
                    end = t if k < t <= hi + 1 else (hi + 1 if t == lo else k + 1)
                    skipped.update(j for j in range(k + 1, end) if ins[j][1].startswith("v_"))
                skip = len(skipped)
                rec = {"kernel": syms[0], "samples_per_iteration": samples, "valu_per_iteration": valu,
                       "valu_per_sample": valu / samples,
                       "valu_per_transparent_sample": (valu - skip) / samples,
                       "salu_per_sample": sum(op.startswith("s_") for op in body) / samples,
                       "vmem_per_sample": loads / samples,
                       "lds_per_sample": sum(op.startswith("ds_") for op in body) / samples,
                       "instructions_per_iteration": len(body)}
                if best is None or rec["valu_per_sample"] < best["valu_per_sample"]:
                    best = rec
            return best
    return None


if __name__ == "__main__":
    import json
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    kind = int(sys.argv[1]) if len(sys.argv) > 1 else 6
    layout = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    print(json.dumps(loop_profile(os.path.join(here, "librtvol.so"), kind, layout)))
