"""Throughput of the PLIC hot path on one MI355X.

One step = one pass of the whole path over resident synthetic inputs:
  * plic_offset forward on N = 2^26 problems with each of the four solvers
    (analytic, optimized SZ, Newton-Raphson, nested intervals), FP32;
  * plic_volume on the same problems (the round trip V0(n, d0(n, V0)));
  * plic_offset backward (optimized SZ), upstream gradient N(0, 1);
  * plic_curvature forward and backward on a 256^3 lattice holding a sphere of
    radius 40 (8^3 supersampled fill levels), FP32 points with FP64 fit.
Each kernel is bracketed by HIP events on the stream it runs on; the step time
is taken around the whole step after a device synchronisation.

Prints one JSON line: value = PLIC solves per second of step time, counting
the 4 N forward solves and the N solves recomputed by the backward (5 N per
step).  Beside it: per-kernel rates with their fraction of the HBM peak and of
the measured VALU issue ceiling (valu_ceiling: a probe of each instruction's
issue rate), the roofline of the dominant kernel, the differentiation
workload (offset forward + backward on 2^24 problems, curvature forward +
backward on a 192^3 perturbed sphere), secondary variants, the paper-method
benchmark, and the CPU-baseline leg.  That leg is the only part that runs
the oracle: its rate on all host cores and on one, the oracle curvature's
rate on the lattice, each solver's error against it, and the precision study
(2^24 near-degenerate problems and the lattice through every precision mode,
with time and error against the oracle).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
VALU_PEAK_TOPS = 39.3          # 256 CU x 64 lanes x 2.4 GHz, non-packed lane-ops / s (x1e12)
METRIC = "PLIC solves/s + curvature cells/s at 1 GPU, fwd+bwd, err vs FP64 oracle"
SOLVERS = ("analytic", "sz", "newton", "nested")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20,
                    help="untimed steps first; the GPU's clock reaches its steady value under this load "
                         "only after about 20 (some 40 ms), and the instruction-bound solvers run up to "
                         "16%% slower before that")
    ap.add_argument("--log2n", type=int, default=26, help="log2 of the PLIC batch size")
    ap.add_argument("--lattice", type=int, default=256)
    ap.add_argument("--radius", type=float, default=40.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paper-isolated", action="store_true",
                    help="skip the compute-isolated timing after the paper's Table 3 method")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the oracle CPU baseline sample")
    ap.add_argument("--only", default="", help="comma list of kernels to run (profiling aid)")
    ap.add_argument("--write-traffic-profile", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM traffic summary from two rocprofv3 --pmc runs and exit (no GPU); "
                         "run it on the tree that was profiled, since it records that tree's kernel source hash")
    ap.add_argument("--traffic-out", default=TRAFFIC_PROFILE, help="where --write-traffic-profile writes")
    ap.add_argument("--write-issue-profile", metavar="SQ_CSV",
                    help="write the instruction-issue summary from a rocprofv3 --pmc run and exit (no GPU)")
    ap.add_argument("--issue-out", default=ISSUE_PROFILE, help="where --write-issue-profile writes")
    ap.add_argument("--write-isa-profile", action="store_true",
                    help="static gfx950 instruction counts of the paper-method benchmark kernels "
                         "(compiles plic_bench.hip to assembly; no GPU)")
    ap.add_argument("--isa-out", default=ISA_PROFILE, help="where --write-isa-profile writes")
    ap.add_argument("--write-valu-profile", metavar="OUT_MD",
                    help="run only the VALU issue-rate probe (GPU) and write its table to OUT_MD")
    ap.add_argument("--write-trace-profile", metavar="TRACE_CSV",
                    help="summarise a rocprofv3 --kernel-trace run of this script (its "
                         "*_kernel_trace.csv) into --trace-out")
    ap.add_argument("--trace-out", default=None, help="where --write-trace-profile writes")
    return ap.parse_args()


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_2p26_problems_256cube_sphere_pmc.md")
ISA_PROFILE = os.path.join(ROOT, "profiles", "isolated_plic_isa_counts_gfx950.md")
# Table 3 (Titan Xp, PTX): arithmetic operations N_a and branches N_b per PLIC, blank run subtracted
PAPER_TABLE3_OPS = {"sz": (132, 12), "sz_kawano": (149, 14), "analytic": (189, 13), "newton": (256, 11),
                    "nested": (106, 13)}
KERNEL_SOURCES = ("plic_math.hpp", "plic_host.hpp", "plic_offset.hip", "plic_curvature.hip")


def code_text(src):
    """C++ source without comments and blank space (string literals kept)"""
    import re
    tok = re.compile(r'"(?:\\.|[^"\\])*"|\'(?:\\.|[^\'\\])*\'|//[^\n]*|/\*.*?\*/', re.S)
    code = tok.sub(lambda m: m.group(0) if m.group(0)[0] in "\"'" else " ", src)
    return "\n".join(" ".join(line.split()) for line in code.splitlines() if line.strip())


def kernel_source_hash():
    """sha256 over the device sources' code (comments and blank space removed,
    so a comment-only edit keeps a measurement valid), in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2006_12838_amd", "csrc", name)) as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of a bench kernel from the committed profiler
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's counters), or
    None when the summary is missing or the kernel sources changed since."""
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    import re
    m = re.search(r"kernel source sha256: `([0-9a-f]{64})`", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(r"^\| " + re.escape(kernel) + r" \| [^|]* \| ([0-9,]+) \|", text, flags=re.M)
    return int(m.group(1).replace(",", "")) if m else None


def measured_issue(kernel):
    """Wavefronts and instructions per wavefront (all VALU, F32 and F64
    transcendentals) of one launch of a bench kernel from the committed
    issue-counter summary, or None when it is missing or the kernel sources
    changed since."""
    try:
        text = open(ISSUE_PROFILE).read()
    except OSError:
        return None
    import re
    m = re.search(r"kernel source sha256: `([0-9a-f]{64})`", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(r"^\| " + re.escape(kernel) + r" \| ([0-9,]+) \| ([0-9.]+) \| ([0-9.]+) \| ([0-9.]+) \|",
                  text, flags=re.M)
    if not m:
        return None
    return {"waves": int(m.group(1).replace(",", "")), "valu": float(m.group(2)), "trans_f32": float(m.group(3)),
            "trans_f64": float(m.group(4))}


def write_valu_profile(out):
    """The VALU probe on its own, at two loop lengths (the difference of the
    two removes the launch and the chains' set-up), as a profile table."""
    import torch

    import paper_2006_12838_amd as P

    dev = torch.device("cuda:0")
    a = valu_ceiling(P, torch, dev, iters=200)
    b = valu_ceiling(P, torch, dev, iters=800)
    lines = [
        "# VALU issue rates on gfx950 (MI355X): plic_bench_valu",
        "",
        "Command (from the repository root on an MI355X, ROCm 7.2):",
        "",
        "```",
        "python3 bench.py --write-valu-profile profiles/valu_ceiling_gfx950.md",
        "```",
        "",
        "2^20 threads (16 waves per SIMD), each issuing 32 x iters instructions of one kind in 8 independent "
        "dependency chains with nothing else in the loop (checked in the kernel's ISA), timed with HIP "
        "events against an iters = 0 launch, after a 10-launch warm-up of the clock.  Cycles per wavefront "
        "instruction are at the nominal 2.4 GHz (1024 SIMDs).",
        "",
        "| instruction | lane-ops/s (iters 200) | lane-ops/s (iters 800) | cycles per wave instruction |",
        "|---|---:|---:|---:|",
    ]
    names = {"fma_f32": "`v_fma_f32`", "fma_f64": "`v_fma_f64`", "sqrt_f32": "`v_sqrt_f32`",
             "rsq_f32": "`v_rsq_f32`", "rcp_f32": "`v_rcp_f32`", "sin_f32": "`v_sin_f32`",
             "exp_f32": "`v_exp_f32`", "log_f32": "`v_log_f32`", "rcp_f64": "`v_rcp_f64`",
             "sqrt_f64": "`v_sqrt_f64`", "fma_sin_f32": "16 `v_fma_f32` + 16 `v_sin_f32`"}
    for op in a:
        lines.append(f"| {names.get(op, op)} | {a[op]['lane_ops_per_s']:.3g} | {b[op]['lane_ops_per_s']:.3g} | "
                     f"{b[op]['cycles_per_wave_instr_at_2p4GHz']:.2f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return out


def valu_bound_ms(issue, ceiling):
    """Time the launch's VALU instructions need at the measured issue rates
    (non-transcendental ones at the v_fma_f32 rate, transcendentals at the
    slowest probed F32 / F64 transcendental's), in ms."""
    trans32 = min(ceiling[k]["lane_ops_per_s"] for k in ("sqrt_f32", "rsq_f32", "rcp_f32", "sin_f32",
                                                          "exp_f32", "log_f32"))
    trans64 = min(ceiling[k]["lane_ops_per_s"] for k in ("rcp_f64", "sqrt_f64"))
    lanes = issue["waves"] * 64
    plain = issue["valu"] - issue["trans_f32"] - issue["trans_f64"]
    return 1e3 * lanes * (plain / ceiling["fma_f32"]["lane_ops_per_s"] + issue["trans_f32"] / trans32
                          + issue["trans_f64"] / trans64)


# bench kernel -> dispatch names (demangled prefixes) that make up one launch
PMC_DISPATCHES = {
    "offset_analytic": ("k_offset<0, float, float, float, 4,",),
    "offset_sz": ("k_offset<1, float, float, float, 4,",),
    "offset_newton": ("k_offset<2, float, float, float, 4,",),
    "offset_nested": ("k_offset<3, float, float, float, 4,",),
    "volume": ("k_volume<float, float, 4>",),
    "offset_backward_sz": ("k_offset_bwd<1, float, float, float, 4,",),
    "curvature_fwd": ("k_curv_scan<true, true>", "k_curv_quads<0, float, double, double, false, 0, false>"),
    "curvature_bwd": ("k_curv_scan<true, false>", "k_curv_quads<0, float, double, double, true, 0, false>",
                      "k_curv_dilate", "k_curv_prefix", "k_curv_gather_direct",
                      "k_curv_gather_fallback<0, float, double, double, 0>"),
    "copy": ("__amd_rocclr_copyBuffer",),
}
ALGORITHMIC_BYTES = {"offset_analytic": 20, "offset_sz": 20, "offset_newton": 20, "offset_nested": 20,
                     "volume": 20, "offset_backward_sz": 36, "curvature_fwd": 8, "curvature_bwd": 8, "copy": 8}


def write_traffic_profile(fetch_csv, write_csv, log2n, lattice, out=TRAFFIC_PROFILE):
    """Summary of two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, in KiB
    per dispatch) of `bench.py --only <kernels>,copy --steps 1 --warmup 0`:
    HBM bytes per launch of each bench kernel, both counters scaled by what
    they read for a plain copy of 4 * 2^log2n bytes."""
    import csv

    def per_dispatch(path):
        acc = {}
        for r in csv.DictReader(open(path)):
            name = r["Kernel_Name"].replace("plic::(anonymous namespace)::", "").replace("void ", "")
            for k, pats in PMC_DISPATCHES.items():
                for pat in pats:
                    if name.startswith(pat):
                        acc.setdefault((k, pat), []).append(float(r["Counter_Value"]))
        return {key: sum(v) / len(v) for key, v in acc.items()}

    fetch, write = per_dispatch(fetch_csv), per_dispatch(write_csv)
    n = 1 << log2n
    cp = ("copy", PMC_DISPATCHES["copy"][0])
    ff, fw = 4 * n / 1024 / fetch[cp], 4 * n / 1024 / write[cp]
    units = {k: (lattice ** 3 if k.startswith("curvature") else n) for k in PMC_DISPATCHES}
    lines = [
        f"# HBM traffic per launch: 2^{log2n} PLIC problems and a {lattice}^3 sphere lattice (R = 40)",
        "",
        "Commands (from the repository root on an MI355X, ROCm 7.2), one counter per run:",
        "",
        "```",
        "# $REPO: the repository root; $OUT: a directory for the profiler's output",
        "cd /tmp && export TMPDIR=/tmp",
        "K=" + ",".join(PMC_DISPATCHES),
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/pmc_FETCH_SIZE -o pmc -- "
        "python3 $REPO/bench.py --only $K --steps 1 --warmup 0 --no-cpu-baseline",
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/pmc_WRITE_SIZE -o pmc -- "
        "python3 $REPO/bench.py --only $K --steps 1 --warmup 0 --no-cpu-baseline",
        "python3 $REPO/bench.py --write-traffic-profile $OUT/pmc_FETCH_SIZE/pmc_counter_collection.csv "
        "$OUT/pmc_WRITE_SIZE/pmc_counter_collection.csv --traffic-out <this file>",
        "```",
        "",
        f"Calibration: a plain device copy of {4 * n:,} bytes (`copy`, torch's `copy_`) reads "
        f"FETCH_SIZE = {fetch[cp]:,.1f} KiB and WRITE_SIZE = {write[cp]:,.1f} KiB, so FETCH_SIZE is scaled "
        f"by {ff:.4f} and WRITE_SIZE by {fw:.4f}.  HBM bytes = 1024 (FETCH_SIZE * {ff:.4f} + "
        f"WRITE_SIZE * {fw:.4f}), summed over the dispatches of one launch.",
        "",
        f"kernel source sha256: `{kernel_source_hash()}` (of the sources' code, comments and blank space removed; "
        f"bench.py reports these bytes as "
        "`roofline.traffic` only while the device sources hash to this value)",
        "",
        "| bench kernel | dispatches | HBM bytes per launch | FETCH_SIZE KiB | WRITE_SIZE KiB | algorithmic bytes | ratio |",
        "|---|---|---:|---:|---:|---:|---:|",
    ]
    for k, pats in PMC_DISPATCHES.items():
        # the dispatches of the launch that ran (the backward that reuses the
        # forward's scan has none; lattices of at most 256 x 256 tiles run no
        # second prefix pass)
        pats = tuple(p for p in pats if (k, p) in fetch and (k, p) in write)
        if not pats:
            continue
        f = sum(fetch[(k, p)] for p in pats)
        w = sum(write[(k, p)] for p in pats)
        hbm = int(round(1024 * (f * ff + w * fw)))
        alg = ALGORITHMIC_BYTES[k] * units[k]
        lines.append(f"| {k} | {' + '.join('`' + p + '`' for p in pats)} | {hbm:,} | {f:,.1f} | {w:,.1f} | "
                     f"{alg:,} | {hbm / alg:.3f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return out


ISSUE_PROFILE = os.path.join(ROOT, "profiles", "valu_issue_2p26_problems_256cube_sphere_pmc.md")
ISSUE_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VALU_TRANS_F32", "SQ_INSTS_VALU_TRANS_F64",
                  "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES")


# instructions that are neither arithmetic nor a branch: waits, memory, control
_NON_ARITH = ("s_waitcnt", "s_endpgm", "s_nop", "s_load", "s_buffer", "s_barrier", "s_setpc", "s_getpc",
              "s_swappc", "s_sleep", "s_dcache", "s_setprio", "s_trap", "s_sendmsg", "s_delay", "s_clause",
              "global_", "buffer_", "flat_", "scratch_", "ds_")


def isa_counts(asm):
    """static instruction counts of each k_isolated<solver, blank> in gfx950
    assembly: arithmetic (vector and scalar ALU, compares and selects
    included), branches, transcendental vector ops"""
    import re
    out, cur = {}, None
    for line in asm.splitlines():
        m = re.match(r"^(_Z\w*k_isolatedILi(\d)ELb(\d)E\w*):", line)
        if m:
            cur = (int(m.group(2)), bool(int(m.group(3))))
            out[cur] = {"arith": 0, "branch": 0, "trans": 0, "total": 0}
            continue
        if cur is None:
            continue
        if line.startswith(".Lfunc_end"):
            cur = None
            continue
        if not line.startswith("\t") or line.strip().startswith((".", ";")):
            continue
        op = line.split()[0]
        c = out[cur]
        c["total"] += 1
        if op.startswith(("s_cbranch", "s_branch")):
            c["branch"] += 1
        elif op.startswith(_NON_ARITH):
            pass
        elif op.startswith(("v_", "s_")):
            c["arith"] += 1
            if re.match(r"v_(sin|cos|rcp|rsq|sqrt|log|exp)_", op):
                c["trans"] += 1
    return out


def write_isa_profile(out_path=ISA_PROFILE):
    """Markdown summary of the static instruction counts of the paper-method
    benchmark kernels, blank run subtracted as in Table 3 (N_a, N_b)."""
    import importlib.util
    import subprocess
    import tempfile
    spec = importlib.util.spec_from_file_location("_plic_build", os.path.join(ROOT, "paper_2006_12838_amd", "_build.py"))
    bld = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bld)
    src = os.path.join(ROOT, "paper_2006_12838_amd", "csrc", "plic_bench.hip")
    with tempfile.TemporaryDirectory() as tmp:
        asm_path = os.path.join(tmp, "plic_bench.s")
        cmd = [bld.HIPCC, *bld.FLAGS, "--offload-device-only", "-S", src, "-o", asm_path]
        subprocess.run(cmd, check=True, capture_output=True)
        counts = isa_counts(open(asm_path).read())
    names = {0: "analytic", 1: "sz", 2: "newton", 3: "nested", 4: "sz_kawano"}
    blank = counts[(1, True)]
    lines = [
        "# Static gfx950 instruction counts of the paper-method benchmark kernels (Table 3's N_a, N_b)",
        "",
        "Command (repository root, no GPU needed):",
        "",
        "```",
        "python3 bench.py --write-isa-profile",
        "# compiles paper_2006_12838_amd/csrc/plic_bench.hip with the library's flags:",
        "# " + " ".join(["hipcc", *bld.FLAGS, "--offload-device-only", "-S", "plic_bench.hip"]),
        "```",
        "",
        f"kernel source sha256: `{kernel_source_hash()}` (of the sources' code, comments and blank space removed)",
        "",
        "Each `k_isolated<solver, false>` inlines one inversion and one forward volume per loop trip; the "
        "blank kernel (`k_isolated<1, true>`, d0 = V0 - 1/2) holds everything else, so the solver's own "
        "static count is the difference, as Table 3 counts PTX with the blank run subtracted.  "
        "`N_a` = vector and scalar ALU instructions (compares, selects and bit operations included; "
        "memory, waits and control excluded), `N_b` = branch instructions; static counts, so a loop "
        "body counts once and an unrolled loop in full.",
        "",
        "| solver | N_a (gfx950) | N_b (gfx950) | transcendental | instructions in the kernel | N_a (Titan Xp PTX) | N_b (PTX) |",
        "|---|---:|---:|---:|---:|---:|---:|",
    ]
    for sv in (1, 4, 0, 2, 3):
        c = counts[(sv, False)]
        pa, pb = PAPER_TABLE3_OPS[names[sv]]
        lines.append(f"| {names[sv]} | {c['arith'] - blank['arith']} | {c['branch'] - blank['branch']} | "
                     f"{c['trans'] - blank['trans']} | {c['total']} | {pa} | {pb} |")
    lines.append(f"| blank (subtracted) | {blank['arith']} | {blank['branch']} | {blank['trans']} | {blank['total']} | – | – |")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return out_path


TRACE_PROFILE = os.path.join(ROOT, "profiles", "hot_path_2p26_problems_256cube_sphere_kernel_trace.md")


def short_kernel_name(name):
    n = name.replace("plic::(anonymous namespace)::", "").replace("void ", "")
    n = n.split("(", 1)[0] if not n.startswith("__amd") else n
    return n[:60]


def write_trace_profile(trace_csv, out=None):
    """Summary of `rocprofv3 --kernel-trace` over the default bench command
    (its *_kernel_trace.csv): per kernel and launch size, the calls, average
    and minimum dispatch time, and the registers and LDS of the dispatch."""
    import csv

    out = out or TRACE_PROFILE
    acc = {}
    for r in csv.DictReader(open(trace_csv)):
        key = (short_kernel_name(r["Kernel_Name"]), int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) *
               int(r["Grid_Size_Z"]))
        d = acc.setdefault(key, {"t": [], "vgpr": r["VGPR_Count"], "agpr": r.get("Accum_VGPR_Count", "0"),
                                 "lds": r["LDS_Block_Size"], "scratch": r["Scratch_Size"],
                                 "wg": r["Workgroup_Size_X"]})
        d["t"].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(d["t"]) for d in acc.values()) or 1.0
    rows = sorted(acc.items(), key=lambda kv: -sum(kv[1]["t"]))
    lines = [
        "# Kernel time, whole hot path: 2^26 PLIC problems and a 256^3 sphere lattice (R = 40)",
        "",
        "Command (from the repository root on an MI355X, ROCm 7.2):",
        "",
        "```",
        "# $REPO: the repository root; $OUT: a directory for the profiler's output",
        "cd /tmp && export TMPDIR=/tmp",
        "rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/prof -o bench -- "
        "python3 $REPO/bench.py --gpus 1 --steps 20 --warmup 5 --no-cpu-baseline",
        "python3 $REPO/bench.py --write-trace-profile $OUT/prof/bench_kernel_trace.csv "
        "--trace-out <this file>",
        "```",
        "",
        f"kernel source sha256: `{kernel_source_hash()}`",
        "",
        "Dispatch durations from the kernel trace, grouped by kernel and launch size (work-items), so the "
        "step's launches (2^26 problems: `k_offset` and `k_volume` at 16,777,216 work-items, `k_offset_bwd` "
        "at 16,777,216) are apart from the same kernels on other sizes (the differentiation workload's "
        "2^24 problems, the precision study).  One bench step launches every step kernel once (5 warm-up "
        "+ 20 timed steps = 25 calls; the counter reset runs once for the forward and once for the "
        "backward, the scan only for the forward: the step's backward reuses it).  The secondary timings after "
        "the timed steps (VALU "
        "probe `k_valu`, plane-sphere, Kawano's SZ, the FP64 solvers, the warm curvature and its variants, "
        "the 192^3 differentiation lattice, the paper-method benchmark `k_isolated`) appear with their own "
        "call counts.",
        "",
        "Template arguments: `k_offset<solver, storage, bulk, cubic, problems per lane, whole blocks>`, "
        "`k_curv_items<solver, points, cubic, fit, backward, normal, neighbour normals>`, "
        "`k_curv_quads<solver, points, cubic, fit, backward, normal, neighbour normals>` (16 lanes per cell), "
        "`k_curv_gather_fallback<solver, points, cubic, fit, normal>`, "
        "`k_curv_gather_direct<neighbour normals, normal, writes the zeros>`; solver 0 analytic, 1 optimized SZ, "
        "2 Newton-Raphson, 3 nested intervals, 4 Kawano's SZ; normal 0 Parker-Youngs.",
        "",
        "| kernel | work-items | calls | avg µs | min µs | share | VGPR | LDS B | scratch B |",
        "|---|---:|---:|---:|---:|---:|---:|---:|---:|",
    ]
    for (name, items), d in rows:
        t = d["t"]
        lines.append(f"| `{name}` | {items:,} | {len(t)} | {sum(t) / len(t):.1f} | {min(t):.1f} | "
                     f"{100 * sum(t) / total:.1f} % | {d['vgpr']} | {d['lds']} | {d['scratch']} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return out


def write_issue_profile(sq_csv, log2n, lattice, out=ISSUE_PROFILE):
    """Summary of one rocprofv3 --pmc run with ISSUE_COUNTERS over
    `bench.py --only <kernels> --steps 1 --warmup 0`: instructions issued per
    wavefront and VALU lane-instructions per unit of work for each bench kernel."""
    import csv

    acc = {}
    for r in csv.DictReader(open(sq_csv)):
        name = r["Kernel_Name"].replace("plic::(anonymous namespace)::", "").replace("void ", "")
        for k, pats in PMC_DISPATCHES.items():
            for pat in pats:
                if name.startswith(pat):
                    d = acc.setdefault(k, {})
                    d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    n = 1 << log2n
    lines = [
        f"# Instruction issue per launch: 2^{log2n} PLIC problems and a {lattice}^3 sphere lattice (R = 40)",
        "",
        "Command (from the repository root on an MI355X, ROCm 7.2):",
        "",
        "```",
        "# $REPO: the repository root; $OUT: a directory for the profiler's output",
        "cd /tmp && export TMPDIR=/tmp",
        "K=" + ",".join(k for k in PMC_DISPATCHES if k != "copy"),
        "rocprofv3 --pmc " + " ".join(ISSUE_COUNTERS) + " --output-format csv -d $OUT/pmc_sq -o pmc -- "
        "python3 $REPO/bench.py --only $K --steps 1 --warmup 0 --no-cpu-baseline",
        "python3 $REPO/bench.py --write-issue-profile $OUT/pmc_sq/pmc_counter_collection.csv "
        "--issue-out <this file>",
        "```",
        "",
        f"kernel source sha256: `{kernel_source_hash()}`",
        "",
        "Counts are per wavefront (64 lanes), summed over the dispatches of one launch; `VALU lane-instr per "
        "unit` = SQ_INSTS_VALU x 64 / units (problems, or lattice cells for the curvature), an upper bound on "
        "the work per unit since inactive lanes count.",
        "",
        "| bench kernel | waves | VALU / wave | of which trans. F32 | trans. F64 | SALU / wave | LDS / wave | "
        "VALU lane-instr per unit | ACTIVE_INST_VALU | BUSY_CYCLES |",
        "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|",
    ]
    for k in PMC_DISPATCHES:
        if k not in acc:
            continue
        c = acc[k]
        w = c.get("SQ_WAVES", 0.0) or 1.0
        units = lattice ** 3 if k.startswith("curvature") else n
        lines.append(f"| {k} | {c.get('SQ_WAVES', 0):,.0f} | {c.get('SQ_INSTS_VALU', 0) / w:.1f} | "
                     f"{c.get('SQ_INSTS_VALU_TRANS_F32', 0) / w:.1f} | {c.get('SQ_INSTS_VALU_TRANS_F64', 0) / w:.1f} | "
                     f"{c.get('SQ_INSTS_SALU', 0) / w:.1f} | {c.get('SQ_INSTS_LDS', 0) / w:.1f} | "
                     f"{c.get('SQ_INSTS_VALU', 0) * 64 / units:.1f} | {c.get('SQ_ACTIVE_INST_VALU', 0):,.0f} | "
                     f"{c.get('SQ_BUSY_CYCLES', 0):,.0f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return out


# Table 3 of the paper (Nvidia Titan Xp, OpenCL, FP32): ps per isolated PLIC and E_avg
# Table 3 (Titan Xp): ps per PLIC and E_avg; None where the paper prints NaN
PAPER_TABLE3 = {"sz": (12.8, 6.58e-8), "analytic": (19.0, 5.73e-8), "newton": (19.2, 5.47e-8),
                "nested": (106.4, 2.86e-8), "sz_kawano": (16.0, None)}
ISOLATED_SOLVERS = SOLVERS + ("sz_kawano",)


def paper_isolated(P, torch, dev, log2n, L=256, reps=64):
    """The paper's GPU benchmark method (Sec. 2.6.2): 2^log2n normals of its mix
    (one axis, one face diagonal, 1/8 random 2D, the rest random 3D), each
    thread sweeping L equally spaced V0 in series with a round trip through the
    forward volume; each variant is run `reps` times (64 in the paper), the
    mean blank-run time (d0 = V0 - 1/2) is subtracted from the mean and the
    difference divided by the N L evaluations.  Context for the paper's
    Table 3, not the headline (which streams inputs from HBM)."""
    import math

    import workloads

    n = 1 << log2n
    t = [torch.from_numpy(a).to(dev) for a in workloads.paper_mix_normals(n, seed=3)]
    err = torch.empty_like(t[0])
    stream = torch.cuda.current_stream(dev)

    def runs(fn):
        """per-run ms of `reps` back-to-back runs after one warm-up run"""
        fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(stream)
        for k in range(reps):
            fn()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]
        mean = sum(ms) / reps
        std = math.sqrt(sum((x - mean) ** 2 for x in ms) / max(reps - 1, 1))
        return mean, std

    blank_ms, blank_sd = runs(lambda: P.plic_bench_isolated_f32(*t, err, L, "sz", True))
    out = {"normals": n, "L": L, "reps": reps, "blank_ms": round(blank_ms, 4), "solvers": {}}
    for s in ISOLATED_SOLVERS:
        ms, sd = runs(lambda: P.plic_bench_isolated_f32(*t, err, L, s, False))
        e = err.double()
        fin = torch.isfinite(e)
        nan_normals = int((~fin).sum().item())
        e_fin = e[fin].sum().item() / (int(fin.sum().item()) * L)
        ps = (ms - blank_ms) * 1e9 / (n * L)
        ps_sd = math.sqrt(sd * sd + blank_sd * blank_sd) * 1e9 / (n * L)
        # E_avg over every evaluation is NaN when any is (JSON null), as the paper prints for Kawano's form
        out["solvers"][s] = {"ms": round(ms, 4), "ps_per_plic": round(ps, 3), "ps_std": round(ps_sd, 3),
                             "E_avg": e_fin if nan_normals == 0 else None, "nan_normals": nan_normals,
                             "E_avg_finite_normals": e_fin,
                             "paper_titan_xp_ps": PAPER_TABLE3[s][0], "paper_E_avg": PAPER_TABLE3[s][1]}
        print(f"bench: isolated {s}: {ps:.3f} +- {ps_sd:.3f} ps/PLIC", file=sys.stderr, flush=True)
    return out


def timed_reps(torch, stream, fn, reps=10):
    """average ms of fn over reps back-to-back calls, HIP events on its stream"""
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def f64_rates(P, torch, tn):
    """The four solvers with FP64 storage and arithmetic on the step's 2^26
    problems (40 bytes per problem), outside the step."""
    t64 = [t.double() for t in tn[:4]]
    out = torch.empty_like(t64[3])
    stream = torch.cuda.current_stream(out.device)
    res = {}
    for s in SOLVERS:
        ms = timed_reps(torch, stream, lambda: P.plic_offset_f64(*t64, out, s))
        n = out.numel()
        gbs = 40 * n / (ms * 1e-3) / 1e9
        res[s] = {"ms": round(ms, 4), "rate": n / (ms * 1e-3), "unit": "solves/s", "GBps": gbs,
                  "hbm_frac": gbs / HBM_PEAK_GBS}
    return res


def curvature_warm(P, torch, tphi, tgk, kap, gphi, ws):
    """Curvature forward and backward repeated back to back: phi (64 MiB at
    256^3) stays in the 256 MB last-level cache, unlike in the step."""
    stream = torch.cuda.current_stream(tphi.device)
    fwd = timed_reps(torch, stream, lambda: P.plic_curvature_f32(tphi, kap, "analytic", "mixed", ws))
    # the workspace holds the forward's scan: the backward that reuses it, then
    # the one that scans phi itself
    bwd = timed_reps(torch, stream, lambda: P.plic_curvature_backward_reuse_f32(tphi, tgk, gphi, "analytic", "mixed",
                                                                                "py", False, ws))
    full = timed_reps(torch, stream, lambda: P.plic_curvature_backward_f32(tphi, tgk, gphi, "analytic", "mixed", ws))
    n = tphi.numel()
    return {"fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4), "bwd_scanning_ms": round(full, 4),
            "fwd_cells_per_s": n / (fwd * 1e-3), "bwd_cells_per_s": n / (bwd * 1e-3)}


def curvature_variants(P, torch, tphi, tgk, kap, gphi, ws):
    """The curvature options beside the base method, on the same 256^3 lattice
    (warm cache, back-to-back calls): the centre-of-mass normal and each
    interface neighbour's own normal (5^3 neighbourhood), forward and backward."""
    stream = torch.cuda.current_stream(tphi.device)
    n = tphi.numel()
    Z, Y, X = tphi.shape
    ws_nbr = torch.empty(P.plic_curvature_workspace_bytes_ex(X, Y, Z, True), dtype=torch.uint8, device=tphi.device)
    res = {}
    for name, fn in (
            ("cm_fwd", lambda: P.plic_curvature_ex_f32(tphi, kap, "analytic", "mixed", "cm", False, ws)),
            ("cm_bwd", lambda: P.plic_curvature_backward_ex_f32(tphi, tgk, gphi, "analytic", "mixed", "cm", False, ws)),
            ("neighbour_normals_fwd",
             lambda: P.plic_curvature_ex_f32(tphi, kap, "analytic", "mixed", "py", True, ws)),
            ("neighbour_normals_bwd",
             lambda: P.plic_curvature_backward_ex_f32(tphi, tgk, gphi, "analytic", "mixed", "py", True, ws_nbr))):
        ms = timed_reps(torch, stream, fn)
        res[name] = {"ms": round(ms, 4), "cells_per_s": n / (ms * 1e-3)}
    return res


def kawano_rate(P, torch, tn, reps=10):
    """Kawano's form of the SZ solution (Sec. 2.4), FP32, on the step's 2^26
    problems: HBM-streamed like the four solvers (20 bytes per problem), timed
    outside the step (a comparison variant, not one of the paper's solvers)."""
    d = torch.empty_like(tn[3])
    stream = torch.cuda.current_stream(d.device)
    P.plic_offset_f32(*tn[:4], d, "sz_kawano", "fp32")
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        P.plic_offset_f32(*tn[:4], d, "sz_kawano", "fp32")
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    n = d.numel()
    gbs = 20 * n / (ms * 1e-3) / 1e9
    return {"ms": round(ms, 4), "rate": n / (ms * 1e-3), "unit": "solves/s", "GBps": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS}


def sphere_rate(P, torch, V0, reps=10):
    """Plane-sphere inversion (Sec. 3) on the same fill levels: HBM-streamed
    V0 -> d0 (8 bytes per problem), outside the step (not a plane-cube solve)."""
    d = torch.empty_like(V0)
    stream = torch.cuda.current_stream(V0.device)
    P.plic_sphere_offset_f32(V0, d)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        P.plic_sphere_offset_f32(V0, d)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    n = V0.numel()
    gbs = 8 * n / (ms * 1e-3) / 1e9
    return {"ms": round(ms, 4), "rate": n / (ms * 1e-3), "unit": "solves/s", "GBps": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(oracle, nx, ny, nz, V0, seconds, chunk):
    """problems/s of the oracle's bisection inverse on chunks of the workload"""
    done, t0, i = 0, time.perf_counter(), 0
    nchunks = max(1, len(V0) // chunk)
    while True:
        s = slice(i * chunk, (i + 1) * chunk)
        oracle.offset(nx[s], ny[s], nz[s], V0[s])
        done += len(V0[s])
        i = (i + 1) % nchunks
        el = time.perf_counter() - t0
        if el >= seconds:
            return done, el


def cpu_baseline(nx, ny, nz, V0, seconds, gpu_offset=None, phi=None):
    """The oracle (bisection on the FP64 forward volume), timed on the host
    cores on chunks of the same workload until `seconds` have passed, then on
    one core for a quarter of that; with phi, the oracle's curvature of the
    whole lattice on all cores and on one.  With gpu_offset ((solver,
    precision) -> the GPU's d0 of the whole batch, on the host), the error of
    each solver and precision against the oracle's d0 of the first chunk."""
    import numpy as np
    import oracle

    oracle.build(force=False)
    threads = oracle.num_threads()
    chunk = 1 << 21
    first = np.asarray(oracle.offset(nx[:chunk], ny[:chunk], nz[:chunk], V0[:chunk]), dtype=np.float64)
    done, el = _oracle_rate(oracle, nx, ny, nz, V0, seconds, chunk)
    oracle.set_num_threads(1)
    try:
        done1, el1 = _oracle_rate(oracle, nx, ny, nz, V0, seconds / 4, 1 << 16)
        curv1 = None
        if phi is not None:
            t0 = time.perf_counter()
            oracle.curvature(phi)
            curv1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(threads)
    out = {"value": done / el, "unit": "PLIC solves/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{done} problems of the 2^{int(math.log2(len(V0)))} workload "
                     f"(chunks of 2^21) through the FP64 oracle's bisection inverse, "
                     f"{el:.1f} s, {threads} OpenMP threads",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "one_core": {"value": done1 / el1, "unit": "PLIC solves/s", "cores": 1,
                        "sample": f"{done1} problems (chunks of 2^16), {el1:.1f} s"}}
    if phi is not None:
        t0 = time.perf_counter()
        k = oracle.curvature(phi)
        curv = time.perf_counter() - t0
        n_if = int(np.count_nonzero(k))
        out["curvature"] = {
            "lattice": list(phi.shape), "interface_cells": n_if,
            "sample": "the oracle's curvature of the whole lattice (bisection offsets, FP64 fit), one call",
            "all_cores": {"s": round(curv, 3), "cells_per_s": phi.size / curv,
                          "interface_cells_per_s": n_if / curv, "cores": threads},
            "one_core": {"s": round(curv1, 3), "cells_per_s": phi.size / curv1,
                         "interface_cells_per_s": n_if / curv1, "cores": 1}}
    if gpu_offset is not None:
        n = len(first)
        err = {}
        for solver in SOLVERS:
            for prec in ("fp32", "mixed"):
                diff = np.abs(np.asarray(gpu_offset(solver, prec)[:n], dtype=np.float64) - first)
                err[f"{solver}/{prec}"] = {"max_abs": float(diff.max()), "rms": float(np.sqrt(np.mean(diff * diff)))}
        out["error_vs_oracle"] = {"quantity": "d0, FP32 storage", "problems": n,
                                  "sample": f"the first {n} problems of the workload", "tolerance": 1e-5,
                                  "per_solver": err}
    return out


def _stats(err):
    import numpy as np

    err = np.asarray(err, dtype=np.float64)
    return {"max_abs": float(err.max()), "rms": float(np.sqrt(np.mean(err * err)))}


def precision_study(P, torch, dev, log2n=24, lattice=None, radius=40.0, step_inputs=None):
    """The precision modes against the oracle (part of the CPU-baseline leg,
    the only part of this script that runs the oracle): 2^log2n near-degenerate
    problems (normals within 1e-4 rad of the axes and diagonals, fill levels
    within 1e-6 of 0, 1 and the case-boundary volumes) through every solver in
    FP32, mixed, FP64 arithmetic with FP32 storage, and FP64 storage, each with
    its time and max / RMS |d0 - oracle|; the step's own random problems in
    FP32 and mixed (time, beside their error in error_vs_oracle); and the
    curvature of the lattice in each mode, with max / RMS |kappa - oracle| over
    the well-conditioned interface cells."""
    import numpy as np
    import oracle
    import workloads

    n = 1 << log2n
    nx, ny, nz, V0 = workloads.near_degenerate_problems(oracle.volume, n, seed=11)
    ref = oracle.offset(nx, ny, nz, V0)
    t32 = [torch.from_numpy(a).to(dev) for a in (nx, ny, nz, V0)]
    t64 = [t.double() for t in t32]
    o32, o64 = torch.empty_like(t32[3]), torch.empty_like(t64[3])
    stream = torch.cuda.current_stream(dev)
    rows = {}
    for solver in SOLVERS:
        for mode in ("fp32", "mixed", "fp64", "f64"):
            if mode == "f64":
                fn, out, bpp = (lambda: P.plic_offset_f64(*t64, o64, solver)), o64, 40
            else:
                fn, out, bpp = (lambda: P.plic_offset_f32(*t32, o32, solver, mode)), o32, 20
            ms = timed_reps(torch, stream, fn, reps=5)
            d = out.cpu().numpy().astype(np.float64)
            rows[f"{solver}/{mode}"] = {"ms": round(ms, 4), "solves_per_s": n / (ms * 1e-3),
                                        "hbm_frac": n * bpp / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                        **_stats(np.abs(d - ref))}
    res = {"problems": {"count": n, "workload": "near-degenerate: normals within 1e-4 rad of the 6 axis, "
                                                "12 face-diagonal and 8 space-diagonal directions; V0 within "
                                                "1e-6 of 0, 1 or a case-boundary volume",
                        "tolerance": {"fp32_storage": 1e-5, "f64": 1e-12}, "per_mode": rows}}
    if step_inputs is not None:
        # the step's own 2^26 random problems: FP32 against mixed, time only
        # (their error against the oracle is error_vs_oracle of the CPU leg)
        tn, out = step_inputs, torch.empty_like(step_inputs[3])
        rand = {}
        for solver in SOLVERS:
            for mode in ("fp32", "mixed"):
                ms = timed_reps(torch, stream, lambda: P.plic_offset_f32(*tn[:4], out, solver, mode), reps=5)
                rand[f"{solver}/{mode}"] = {"ms": round(ms, 4)}
            rand[f"{solver}/mixed"]["mixed_over_fp32"] = round(rand[f"{solver}/mixed"]["ms"] /
                                                               rand[f"{solver}/fp32"]["ms"], 3)
        res["random_problems"] = {"count": int(tn[3].numel()), "per_mode": rand}
    for solver in SOLVERS:
        rows[f"{solver}/mixed"]["mixed_over_fp32"] = round(rows[f"{solver}/mixed"]["ms"] /
                                                           rows[f"{solver}/fp32"]["ms"], 3)
    if lattice is not None:
        phi = lattice
        kref, flags = oracle.curvature(phi, flags=True)
        cells = np.flatnonzero(flags & 1)
        _, info = oracle.curvature_cells(phi, cells)
        good = cells[(info[:, 0] >= 5) & (info[:, 2] <= 1e6)]
        kr = kref.ravel()[good]
        tp = torch.from_numpy(phi).to(dev)
        k = torch.empty_like(tp)
        Z, Y, X = phi.shape
        ws = torch.empty(P.plic_curvature_workspace_bytes(X, Y, Z), dtype=torch.uint8, device=dev)
        crow = {}
        for mode in ("fp32", "mixed", "fp64"):
            ms = timed_reps(torch, stream, lambda: P.plic_curvature_f32(tp, k, "analytic", mode, ws), reps=5)
            kg = k.cpu().numpy().ravel()[good].astype(np.float64)
            crow[mode] = {"fwd_ms": round(ms, 4), "cells_per_s": phi.size / (ms * 1e-3),
                          **_stats(np.abs(kg - kr)), "max_abs_times_R": float(np.abs(kg - kr).max() * radius),
                          "mean_kappa_R": float(kg.mean() * radius)}
        res["curvature"] = {"lattice": list(phi.shape), "cells_compared": int(good.size),
                            "interface_cells": int(cells.size),
                            "compared": "interface cells with >= 5 points and pivot ratio <= 1e6 "
                                        "(analytic points; warm cache)",
                            "tolerance": "|dk| <= 1e-5 + 1e-3 |k| per cell (FP64 fit)", "per_mode": crow}
    return res


def differentiation(P, torch, dev, tn, log2n=24):
    """Forward + backward timings of the differentiation workload: plic_offset
    on the first 2^log2n problems of the step (upstream N(0,1)), and the
    curvature of a 192^3 perturbed sphere (R = 50, l <= 6 harmonics, 5 %
    amplitude) with N(0,1) upstream on every interface cell, FP32 points and
    FP64 fit.  Warm back-to-back calls."""
    import numpy as np
    import workloads

    n = 1 << log2n
    t = [x[:n] for x in tn]
    d0 = torch.empty_like(t[3])
    g = [torch.empty_like(t[3]) for _ in range(4)]
    stream = torch.cuda.current_stream(dev)
    fwd = timed_reps(torch, stream, lambda: P.plic_offset_f32(*t[:4], d0, "sz", "fp32"))
    bwd = timed_reps(torch, stream, lambda: P.plic_offset_backward_f32(*t[:4], t[4], *g, "sz", "fp32"))
    res = {"plic_offset": {"problems": n, "solver": "sz", "precision": "fp32", "fwd_ms": round(fwd, 4),
                           "bwd_ms": round(bwd, 4), "fwd_bwd_solves_per_s": n / ((fwd + bwd) * 1e-3),
                           "bytes_per_problem": 56,
                           "hbm_frac": n * 56 / ((fwd + bwd) * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    phi, _, _ = workloads.perturbed_sphere_lattice(N=192, R=50.0, seed=0)
    iface = (phi > 0) & (phi < 1)
    gk = np.where(iface, workloads.upstream_grad(phi.shape, seed=3), 0.0).astype(np.float32)
    tp, tg = torch.from_numpy(phi).to(dev), torch.from_numpy(gk).to(dev)
    kap, gp = torch.empty_like(tp), torch.empty_like(tp)
    Z, Y, X = phi.shape
    ws = torch.empty(P.plic_curvature_workspace_bytes(X, Y, Z), dtype=torch.uint8, device=dev)
    cf = timed_reps(torch, stream, lambda: P.plic_curvature_f32(tp, kap, "analytic", "mixed", ws))
    cb = timed_reps(torch, stream, lambda: P.plic_curvature_backward_reuse_f32(tp, tg, gp, "analytic", "mixed", "py",
                                                                               False, ws))
    res["curvature"] = {"lattice": [192, 192, 192], "workload": "perturbed sphere R=50, l<=6, 5% amplitude",
                        "interface_cells": int(iface.sum()), "fwd_ms": round(cf, 4), "bwd_ms": round(cb, 4),
                        "fwd_bwd_cells_per_s": phi.size / ((cf + cb) * 1e-3),
                        "bytes_per_cell": 20, "hbm_frac": phi.size * 20 / ((cf + cb) * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return res


def valu_ceiling(P, torch, dev, threads=1 << 20, iters=800):
    """Measured issue rate of each probed VALU instruction (plic_bench_valu:
    32 * iters instructions per thread, minus an empty launch), in lane
    operations per second and in cycles per wavefront instruction at the
    nominal 2.4 GHz."""
    from paper_2006_12838_amd._lib import VALU_OPS

    sink = torch.empty(threads, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    for _ in range(10):
        P.plic_bench_valu("fma_f32", sink, 4 * iters)
    res = {}
    for op in VALU_OPS:
        t = timed_reps(torch, stream, lambda: P.plic_bench_valu(op, sink, iters), reps=5)
        t0 = timed_reps(torch, stream, lambda: P.plic_bench_valu(op, sink, 0), reps=5)
        rate = threads * 32 * iters / ((t - t0) * 1e-3)
        res[op] = {"lane_ops_per_s": rate, "cycles_per_wave_instr_at_2p4GHz": 1024 * 2.4e9 / (rate / 64)}
    return res


def main():
    args = parse()
    if args.write_traffic_profile:
        print(write_traffic_profile(*args.write_traffic_profile, args.log2n, args.lattice, args.traffic_out))
        return
    if args.write_isa_profile:
        print(write_isa_profile(args.isa_out))
        return
    if args.write_issue_profile:
        print(write_issue_profile(args.write_issue_profile, args.log2n, args.lattice, args.issue_out))
        return
    if args.write_valu_profile:
        print(write_valu_profile(args.write_valu_profile))
        return
    if args.write_trace_profile:
        print(write_trace_profile(args.write_trace_profile, args.trace_out))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; --gpus must be 1 (the PLIC path has no cross-GPU step)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2006_12838_amd as P
    import workloads

    dev = torch.device("cuda:0")
    N = 1 << args.log2n
    t_gen = time.perf_counter()
    nx, ny, nz, V0 = workloads.plic_problems(N, seed=0)
    gd = workloads.upstream_grad(N, seed=1)
    phi, _ = workloads.sphere_lattice(N=args.lattice, R=args.radius, seed=0)
    gk = workloads.upstream_grad(phi.shape, seed=2)
    print(f"bench: inputs generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)

    tn = [torch.from_numpy(a).to(dev) for a in (nx, ny, nz, V0, gd)]
    d0 = torch.empty_like(tn[3])
    Vb = torch.empty_like(tn[3])
    gout = [torch.empty_like(tn[3]) for _ in range(4)]
    tphi = torch.from_numpy(phi).to(dev)
    tgk = torch.from_numpy(gk).to(dev)
    kap = torch.empty_like(tphi)
    gphi = torch.empty_like(tphi)
    ws = torch.empty(P.plic_curvature_workspace_bytes(*phi.shape[::-1]), dtype=torch.uint8, device=dev)
    cells = phi.size
    n_iface = int(((phi > 0) & (phi < 1)).sum())

    kernels = []  # (name, fn, units, unit_name, algorithmic bytes per unit)
    for s in SOLVERS:
        kernels.append((f"offset_{s}", (lambda s=s: P.plic_offset_f32(*tn[:4], d0, s, "fp32")),
                        N, "solves", 20))
    kernels.append(("volume", lambda: P.plic_volume_f32(tn[0], tn[1], tn[2], d0, Vb, "fp32"), N, "solves", 20))
    kernels.append(("offset_backward_sz",
                    lambda: P.plic_offset_backward_f32(*tn[:4], tn[4], *gout, "sz", "fp32"), N, "solves", 36))
    kernels.append(("curvature_fwd", lambda: P.plic_curvature_f32(tphi, kap, "analytic", "mixed", ws),
                    cells, "cells", 8))
    # the backward follows its forward on the same workspace and reuses its scan
    kernels.append(("curvature_bwd",
                    lambda: P.plic_curvature_backward_reuse_f32(tphi, tgk, gphi, "analytic", "mixed", "py", False, ws),
                    cells, "cells", 8))
    if args.only:
        keep = set(args.only.split(","))
        kernels = [k for k in kernels if k[0] in keep]
        if "copy" in keep:
            # plain device copy of N floats (4 N bytes read, 4 N written): the
            # reference for scaling the HBM byte counters of a profiler run
            csrc = torch.empty(N, dtype=torch.float32, device=dev).uniform_()
            cdst = torch.empty_like(csrc)
            kernels.append(("copy", lambda: cdst.copy_(csrc), N, "floats", 8))

    stream = torch.cuda.current_stream(dev)
    # the VALU probe runs first: its measurement is reported beside the step,
    # and its ~0.1 s of issue-bound work brings the GPU clock up before the
    # warm-up steps (the instruction-bound solvers time up to 16 % slow on a
    # clock still ramping)
    ceiling = None if args.only else valu_ceiling(P, torch, dev)
    # one pair of events per kernel and step: the K steps run back to back,
    # and the per-kernel times are read after the closing synchronize
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in kernels]
          for _ in range(args.steps)]

    def step(pairs):
        for (name, fn, *_), pair in zip(kernels, pairs):
            if pair:
                pair[0].record(stream)
            fn()
            if pair:
                pair[1].record(stream)

    for _ in range(args.warmup):
        step([None] * len(kernels))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(ev[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    per = {k[0]: 0.0 for k in kernels}
    for pairs in ev:
        for (name, *_), (a, b) in zip(kernels, pairs):
            per[name] += a.elapsed_time(b)
    print(f"bench: {args.steps} steps timed", file=sys.stderr, flush=True)

    rates = {}
    for name, fn, units, uname, bpu in kernels:
        ms = per[name] / args.steps
        rates[name] = {"ms": round(ms, 4), "rate": units / (ms * 1e-3), "unit": f"{uname}/s",
                       "GBps": units * bpu / (ms * 1e-3) / 1e9,
                       "hbm_frac": units * bpu / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    solves = sum(N for k in kernels if k[0].startswith("offset_"))
    value = solves / (ms_step * 1e-3)
    dom = max(kernels, key=lambda k: per[k[0]])
    dms = per[dom[0]] / args.steps
    dgbs = dom[2] * dom[4] / (dms * 1e-3) / 1e9
    roofline = {"kernel": dom[0], "bound": "hbm", "achieved": round(dgbs, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(dgbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom[0]),
                "bytes_per_unit": dom[4], "units_per_launch": dom[2]}
    fast = min((k for k in kernels if k[0].startswith("offset_") and k[0] != "offset_backward_sz"),
               key=lambda k: per[k[0]], default=None)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "PLIC solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2^{args.log2n} plane-cube problems (unit Gaussian normals, uniform V0, "
                               f"2% edge cases) x 4 solvers fwd + volume + SZ bwd; "
                               f"{args.lattice}^3 sphere R={args.radius:g} curvature fwd+bwd",
                   "problems": N, "lattice": [args.lattice] * 3, "interface_cells": n_iface,
                   "precision": {"plic": "fp32", "curvature": "mixed (fp32 points, fp64 fit)"}},
        "kernels": rates,
        "curvature_cells_per_s": (cells / ((per.get("curvature_fwd", 0) + per.get("curvature_bwd", 0))
                                           / args.steps * 1e-3)) if "curvature_fwd" in per else None,
        "fastest_solver": None if fast is None else {"solver": fast[0][7:], "solves_per_s": rates[fast[0]]["rate"],
                                                     "hbm_frac": rates[fast[0]]["hbm_frac"]},
        "roofline": roofline,
    }
    if not args.only:
        out["valu_ceiling"] = ceiling
        for name in rates:
            iss = measured_issue(name)
            if iss is None:
                rates[name]["valu_frac"] = None
                continue
            rates[name]["valu_frac"] = round(valu_bound_ms(iss, ceiling) / rates[name]["ms"], 4)
            rates[name]["binds"] = "hbm" if rates[name]["hbm_frac"] >= rates[name]["valu_frac"] else "valu"
        out["differentiation"] = differentiation(P, torch, dev, tn)
        out["sphere_offset"] = sphere_rate(P, torch, tn[3])
        out["offset_sz_kawano"] = kawano_rate(P, torch, tn)
        out["offset_f64"] = f64_rates(P, torch, tn)
        out["curvature_warm"] = curvature_warm(P, torch, tphi, tgk, kap, gphi, ws)
        out["curvature_variants"] = curvature_variants(P, torch, tphi, tgk, kap, gphi, ws)
    if not args.no_paper_isolated and not args.only:
        out["paper_isolated"] = paper_isolated(P, torch, dev, args.log2n)
    if not args.no_cpu_baseline:
        def gpu_offset(solver, prec):
            P.plic_offset_f32(*tn[:4], d0, solver, prec)
            torch.cuda.synchronize()
            return d0[: 1 << 21].cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(nx, ny, nz, V0, args.cpu_seconds, gpu_offset, phi)
        if not args.only:
            out["precision_study"] = precision_study(P, torch, dev, 24, phi, args.radius, tn)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
