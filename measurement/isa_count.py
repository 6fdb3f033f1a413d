"""Count instructions and SIMD issue cycles per pair in the compiled pair
kernels' inner loops.

    python measurement/isa_count.py

Compiles csrc/pair_kernels.hip, csrc/mfma_kernels.hip (FP32 and FP64 matrix-core
kernels), csrc/sym_kernels.hip and csrc/far_field.hip to gfx950 assembly
(the same flags as the library build) and, for each kernel variant, finds the
innermost loop that evaluates the most pairs per trip (the unrolled
steady-state loop; one v_rsq per pair and lane, in the far-field kernels one
phase reduction: v_fract_f64 on the FP32 path, v_rndne_f64 on the FP64 path),
counts its instructions and divides by the pairs per trip (ordered pairs: an
evaluation of the symmetric cell-cell kernel and of the cell-face kernel
counts twice).

Issue-cycle model (SIMD cycles one wave64 instruction occupies; the chip has
256 CUs x 4 SIMDs at 2.4 GHz):
  FP32 and 32-bit integer VALU      2   (157.3 TFLOP/s FP32 = 64 FLOP/cycle/SIMD)
  FP64 and 64-bit integer VALU      4   (78.6 TFLOP/s FP64)
  FP32 transcendental (rsq sin cos) 8   (quarter of the FP32 rate)
  FP64 transcendental (rsq_f64)    16
  v_mfma_f32_16x16x4_f32           32   (2048 FLOP at 64 FLOP/cycle/SIMD)
  v_mfma_f64_16x16x4_f64           64   (2048 FLOP at 78.6 TFLOP/s FP64 matrix = 32 FLOP/cycle/SIMD)
  DPP moves (v_mov_b32_dpp)         4   (measured)
Microbenchmarks on MI355X give 2.5-2.8, 4.4-5.8, 8.5, 16.3, 32.5 and 4.1 cycles
with 8 independent chains per lane, and show matrix-core and VALU time adding
up (no overlap) for FP32.  Writes isa_counts.json beside this file; bench.py
reads it to turn measured pair rates into issue cycles per second.  This is
measurement tooling for the benchmark, not part of the library.
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
sys.path.insert(0, os.path.join(os.path.dirname(HERE), "paper_2607_06429_amd"))
import build as B  # noqa: E402

MODES = {0: "fwd_single_layer", 1: "fwd_double_layers", 2: "adj_double_layers", 3: "source_sums"}


def assemble(src: str) -> str:
    out = os.path.join(tempfile.mkdtemp(), src + ".s")
    cmd = [B._hipcc(), *B.flags_for(src), "--cuda-device-only", "-S",
           os.path.join(B.CSRC, src), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return open(out).read()


def cycles(op: str) -> int:
    """Issue cycles of one wave64 instruction (the model above)."""
    if op.startswith("v_mfma_f64"):
        return 64
    if op.startswith("v_mfma"):
        return 32
    if "_dpp" in op:
        return 4
    if re.match(r"v_(rsq|rcp|sqrt)_f64", op):
        return 16
    if re.match(r"v_(rsq|sin|cos|rcp|sqrt|exp|log)_", op):
        return 8
    if re.search(r"_(f64|u64|i64|b64)", op) or op.startswith("v_mad_u64") or op.startswith("v_mad_i64"):
        return 4
    return 2


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


PAIR_MARK = r"v_rsq"


def kernels(asm: str):
    """(symbol, result key, right-hand sides per trip[, per-pair marker]) of every pair kernel."""
    for nm in re.findall(r"^(_Z\w+far_field_kernel\w+):", asm, re.M):
        cls, R, acc = re.search(r"far_field_kernelILi(\d)ELi(\d+)E(\w)E", nm).groups()
        mark = r"v_fract_f64" if acc == "f" else r"v_rndne_f64"
        yield (nm, "far_field_%s_%s_R%s" % ("single_layer" if cls == "0" else "double_layers",
                                            "fp64" if acc == "d" else "fp32", R), int(R), mark)
    for nm in re.findall(r"^(_Z\w+pair_sum_kernel\w+):", asm, re.M):
        mode, R, acc = re.search(r"kernelILi(\d)ELi(\d+)Ed(\w)", nm).groups()
        yield nm, "%s_%s_R%s" % (MODES[int(mode)], "fp64" if acc == "d" else "fp32", R), int(R)
    for nm in re.findall(r"^(_Z\w+mfma_fwd_kernel\w+):", asm, re.M):
        cls, tg, nb, m3 = re.search(r"kernelILi(\d)ELi(\d)ELi(\d)ELb(\d)E", nm).groups()
        yield nm, "mfma_%s_fp32_tg%s_nb%s%s" % (MODES[int(cls)], tg, nb, "_3m" if m3 == "1" else ""), 16 * int(nb)
    for nm in re.findall(r"^(_Z\w+mfma64_fwd_kernel\w+):", asm, re.M):
        cls, nb, m3 = re.search(r"kernelILi(\d)ELi(\d)ELb(\d)E", nm).groups()
        yield (nm, "mfma64_%s_fp64_nb%s%s" % (MODES[int(cls)], nb, "_3m" if m3 == "1" else ""), 16 * int(nb),
               r"v_rsq_f64")
    for nm in re.findall(r"^(_Z\w+sym_kernel\w+):", asm, re.M):
        g, acc, t, adj = re.search(r"sym_kernelILi(\d)E(\w)Lb(\d)ELb(\d)E", nm).groups()
        if g == "4":   # the default group size; the inner loop is the same for every size
            # T variants: the loop of the items with grad-alpha cells (the most instructions per pair)
            tag = "_t_adj" if adj == "1" else "_t" if t == "1" else ""
            yield nm, "sym_single_layer%s_%s_R1" % (tag, "fp64" if acc == "d" else "fp32"), 1
    for nm in re.findall(r"^(_Z\w+cf_kernel\w+):", asm, re.M):
        acc, t, adj = re.search(r"cf_kernelILi\d+E(\w)Lb(\d)ELb(\d)E", nm).groups()
        tag = ("_t" if t == "1" else "") + ("_adj" if adj == "1" else "")
        yield nm, "cell_face%s_%s_R1" % (tag, "fp64" if acc == "d" else "fp32"), 1


def count(asm: str) -> dict:
    res = {}
    for item in kernels(asm):
        nm, key, R = item[:3]
        mark = item[3] if len(item) > 3 else PAIR_MARK
        i = asm.index(nm + ":")
        lines = asm[i:asm.index(".Lfunc_end", i)].split("\n")
        sym = "sym_kernel" in nm or "cf_kernel" in nm
        best = None
        for a, b in inner_loops(lines):
            body = [x.strip() for x in lines[a:b + 1]
                    if x.strip() and not x.strip().startswith((";", "."))]
            nrsq = sum(1 for x in body if re.match(mark, x))
            if nrsq == 0:
                continue
            if sym:
                # the tile-pair loop (source side carried along: the most DPP moves per pair),
                # not the 63-step loop of a tile with itself; among equals the shortest copy,
                # in a T variant the longest (the loop that adds the adjoint double layer)
                dpp = sum(1 for x in body if "_dpp" in x.split()[0]) / nrsq
                if "_t_" in key:
                    rank = (dpp > 0, len(body) / nrsq)
                else:
                    rank = (dpp, nrsq, -len(body))
                if best is None or rank > best[2]:
                    best = (nrsq, body, rank)
                continue
            # the unrolled steady-state loop evaluates the most pairs per trip
            if best is None or nrsq > best[0] or (nrsq == best[0] and len(body) < len(best[1])):
                best = (nrsq, body)
        if best is None:
            continue
        nrsq, body = best[0], best[1]
        # each evaluation of the symmetric kernel serves two ordered pairs
        per_eval = 2 if sym else 1
        c = collections.Counter()
        for x in body:
            op = x.split()[0]
            if op.startswith("v_"):
                c["cycles"] += cycles(op)
            if op.startswith("v_mfma"):
                c["mfma"] += 1
            elif op.startswith("v_"):
                c["valu"] += 1
                if re.match(r"v_(rsq|sin|cos|rcp|sqrt|exp|log)", op):
                    c["trans"] += 1
                if "_f64" in op:
                    c["f64"] += 1
            elif op.startswith("s_load"):
                c["smem"] += 1
            elif op.startswith("s_"):
                c["salu"] += 1
        res[key] = {"pairs_per_trip": nrsq * per_eval,
                    "rhs_per_trip": R,
                    "cycles_per_pair": c["cycles"] / (64.0 * nrsq * per_eval),
                    "mfma_per_pair": c["mfma"] / nrsq,
                    "valu_per_pair": c["valu"] / nrsq,
                    "f64_per_pair": c["f64"] / nrsq,
                    "trans_per_pair": c["trans"] / nrsq,
                    "salu_per_pair": c["salu"] / nrsq,
                    "smem_per_pair": c["smem"] / nrsq}
    return res


def main():
    res = count(assemble("pair_kernels.hip"))
    res.update(count(assemble("mfma_kernels.hip")))
    res.update(count(assemble("sym_kernels.hip")))
    res.update(count(assemble("far_field.hip")))
    out = os.path.join(HERE, "isa_counts.json")
    with open(out, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    for k in sorted(res):
        print(k, {a: round(b, 2) for a, b in res[k].items()})
    print("wrote", out)


if __name__ == "__main__":
    main()
