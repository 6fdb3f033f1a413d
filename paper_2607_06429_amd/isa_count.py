"""Count VALU instructions per pair in the compiled pair-kernel inner loops.

    python paper_2607_06429_amd/isa_count.py

Compiles csrc/pair_kernels.hip to gfx950 assembly (the same flags as the
library build) and, for each kernel variant, finds the innermost loop that
evaluates the most pairs per trip (the unrolled steady-state loop; one v_rsq
per pair), counts its vector
ALU instructions and divides by the number of pairs per trip (the number of
v_rsq instructions in the loop).  Writes isa_counts.json beside this file;
bench.py reads it to convert measured pair rates into VALU lane-operations.
"""
from __future__ import annotations

import collections
import json
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
import build as B  # noqa: E402

MODES = {0: "fwd_single_layer", 1: "fwd_double_layers", 2: "adj_double_layers", 3: "source_sums"}


def assemble() -> str:
    out = os.path.join(tempfile.mkdtemp(), "pair.s")
    cmd = [B._hipcc(), *B.FLAGS, "--cuda-device-only", "-S",
           os.path.join(B.CSRC, "pair_kernels.hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return open(out).read()


def inner_loops(body_lines):
    """(start, end) line spans of the innermost loops: back-edges grouped by
    their header label, keeping loops that contain no other loop header."""
    labels = {}
    for idx, l in enumerate(body_lines):
        m = re.match(r"^(\.LBB\d+_\d+):", l)
        if m:
            labels[m.group(1)] = idx
    span = {}
    for idx, l in enumerate(body_lines):
        m = re.search(r"s_(?:cbranch_\w+|branch)\s+(\.LBB\d+_\d+)", l)
        if m and m.group(1) in labels and labels[m.group(1)] < idx:
            h = labels[m.group(1)]
            span[h] = max(span.get(h, h), idx)
    loops = sorted(span.items())
    return [(a, b) for a, b in loops
            if not any(a < a2 <= b and (a2, b2) != (a, b) for a2, b2 in loops)]


def count(asm: str) -> dict:
    res = {}
    for nm in re.findall(r"^(_Z\w+pair_sum_kernel\w+):", asm, re.M):
        mode, R, acc = re.search(r"kernelILi(\d)ELi(\d+)Ed(\w)", nm).groups()
        i = asm.index(nm + ":")
        lines = asm[i:asm.index(".Lfunc_end", i)].split("\n")
        best = None
        for a, b in inner_loops(lines):
            body = [x.strip() for x in lines[a:b + 1]
                    if x.strip() and not x.strip().startswith((";", "."))]
            nrsq = sum(1 for x in body if x.startswith("v_rsq"))
            if nrsq == 0:
                continue
            # the unrolled steady-state loop evaluates the most pairs per trip
            if best is None or nrsq > best[0] or (nrsq == best[0] and len(body) < len(best[1])):
                best = (nrsq, body)
        if best is None:
            continue
        nrsq, body = best
        c = collections.Counter()
        for x in body:
            op = x.split()[0]
            if op.startswith("v_"):
                c["valu"] += 1
                if re.match(r"v_(rsq|sin|cos|rcp|sqrt|exp|log)", op):
                    c["trans"] += 1
                if "_f64" in op:
                    c["f64"] += 1
            elif op.startswith("s_load"):
                c["smem"] += 1
            elif op.startswith("s_"):
                c["salu"] += 1
        key = "%s_%s_R%s" % (MODES[int(mode)], "fp64" if acc == "d" else "fp32", R)
        res[key] = {"pairs_per_trip": nrsq,
                    "valu_per_pair": c["valu"] / nrsq,
                    "f64_per_pair": c["f64"] / nrsq,
                    "trans_per_pair": c["trans"] / nrsq,
                    "salu_per_pair": c["salu"] / nrsq,
                    "smem_per_pair": c["smem"] / nrsq}
    return res


def main():
    res = count(assemble())
    out = os.path.join(HERE, "isa_counts.json")
    with open(out, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    for k in sorted(res):
        print(k, {a: round(b, 2) for a, b in res[k].items()})
    print("wrote", out)


if __name__ == "__main__":
    main()
