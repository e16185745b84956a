"""Host logic of bench.py (no GPU): the source hash that ties a profiler
summary to the kernels it measured, the lookup of the measured HBM bytes,
the conversion of the two counter runs into bytes per launch by a plain
copy's counters, the refusal of more than one GPU, and the CPU leg's error
report against the oracle."""
import os
import shutil
import subprocess
import sys

import pytest

import bench


def test_code_text_drops_comments_and_blank_space_only():
    a = 'int f(int x) {  // twice\n    /* a\n       block */ return 2 * x;\n\n}\nconst char* s = "// kept";\n'
    b = 'int f(int x) {\n  return 2 * x;   // other words\n}\nconst char* s = "// kept";\n'
    assert bench.code_text(a) == bench.code_text(b)
    assert '"// kept"' in bench.code_text(a)
    assert bench.code_text(a) != bench.code_text(a.replace("2 * x", "3 * x"))


def copy_sources(tmp_path):
    dst = tmp_path / "paper_2006_12838_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(bench.ROOT, "paper_2006_12838_amd", "csrc", name), dst / name)
    return dst


def test_source_hash_follows_code_not_comments(tmp_path, monkeypatch):
    ref = bench.kernel_source_hash()
    dst = copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == ref
    src = dst / "plic_offset.hip"
    text = src.read_text()
    src.write_text("// a new leading comment\n" + text.replace("\n", "\n\n", 3))
    assert bench.kernel_source_hash() == ref
    src.write_text(text.replace("kBwdBlock = 512", "kBwdBlock = 256", 1))
    assert bench.kernel_source_hash() != ref


def write_profile(path, digest, rows):
    lines = [f"kernel source sha256: `{digest}` (test)", "",
             "| bench kernel | dispatches | HBM bytes per launch | FETCH_SIZE KiB | WRITE_SIZE KiB | algorithmic bytes | ratio |",
             "|---|---|---:|---:|---:|---:|---:|"]
    lines += [f"| {k} | `k` | {v:,} | 1.0 | 1.0 | 1 | 1.000 |" for k, v in rows.items()]
    path.write_text("\n".join(lines) + "\n")


def test_measured_traffic_only_for_the_profiled_sources(tmp_path, monkeypatch):
    prof = tmp_path / "traffic.md"
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    assert bench.measured_traffic("offset_backward_sz") is None                 # no summary
    write_profile(prof, bench.kernel_source_hash(), {"offset_backward_sz": 2415919104, "volume": 7})
    assert bench.measured_traffic("offset_backward_sz") == 2415919104
    assert bench.measured_traffic("volume") == 7
    assert bench.measured_traffic("offset_sz") is None                          # not in the table
    write_profile(prof, "0" * 64, {"offset_backward_sz": 2415919104})
    assert bench.measured_traffic("offset_backward_sz") is None                 # sources changed


def write_counters(path, values):
    lines = ["Kernel_Name,Counter_Value"]
    for name, v in values:
        lines.append(f'"{name}",{v}')
    path.write_text("\n".join(lines) + "\n")


def test_traffic_profile_scales_by_the_copy(tmp_path):
    """FETCH_SIZE that reads half the copy's bytes and WRITE_SIZE that reads
    all of them: each counter is scaled by its own copy factor, dispatches of
    one launch are summed, and repeated dispatches are averaged."""
    log2n, n = 10, 1 << 10
    kib = 4 * n / 1024                                                         # one array of n floats
    fetch = [("__amd_rocclr_copyBuffer", kib / 2),
             ("void plic::(anonymous namespace)::k_offset_bwd<1, float, float, float, 4, true>(...)", 5 * kib / 2),
             ("void plic::(anonymous namespace)::k_offset_bwd<1, float, float, float, 4, true>(...)", 5 * kib / 2)]
    write = [("__amd_rocclr_copyBuffer", kib),
             ("void plic::(anonymous namespace)::k_offset_bwd<1, float, float, float, 4, true>(...)", 4 * kib),
             ("void plic::(anonymous namespace)::k_offset_bwd<1, float, float, float, 4, true>(...)", 4 * kib)]
    fc, wc = tmp_path / "fetch.csv", tmp_path / "write.csv"
    write_counters(fc, fetch)
    write_counters(wc, write)
    out = tmp_path / "traffic.md"
    bench.write_traffic_profile(str(fc), str(wc), log2n, 8, str(out))
    rows = {line.split("|")[1].strip(): line for line in out.read_text().splitlines() if line.startswith("| ")}
    assert "offset_backward_sz" in rows and "copy" in rows
    cells = [c.strip() for c in rows["offset_backward_sz"].split("|")]
    assert int(cells[3].replace(",", "")) == 36 * n                           # 5 reads + 4 writes of 4 B
    assert cells[7] == "1.000"
    assert "volume" not in rows                                               # no dispatches, no row


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_reports_error_against_the_oracle():
    """The CPU leg times the oracle and compares each solver's GPU offsets
    with the oracle's for the first chunk; here a stand-in GPU result is the
    oracle's own plus a known shift."""
    import numpy as np
    import oracle
    import workloads

    nx, ny, nz, V0 = workloads.plic_problems(4096, seed=3)
    ref = np.asarray(oracle.offset(nx, ny, nz, V0), dtype=np.float64)
    shift = {"analytic": 0.0, "sz": 2e-7, "newton": -3e-6, "nested": 1e-5}
    prec_shift = {"fp32": 0.0, "mixed": 1e-6}
    phi, _ = workloads.sphere_lattice(N=16, R=4.0, seed=1)
    out = bench.cpu_baseline(nx, ny, nz, V0, 0.01,
                             lambda s, p: (ref + shift[s] + prec_shift[p]).astype(np.float32), phi)
    assert out["kind"] == "oracle" and out["value"] > 0 and out["cores"] >= 1
    assert out["one_core"]["cores"] == 1 and out["one_core"]["value"] > 0 and out["cpu_model"]
    assert oracle.num_threads() == out["cores"]                         # restored after the one-core run
    cur = out["curvature"]
    assert cur["interface_cells"] == int(np.count_nonzero(oracle.curvature(phi)))
    assert cur["all_cores"]["cells_per_s"] > 0 and cur["one_core"]["cores"] == 1
    err = out["error_vs_oracle"]
    assert err["problems"] == 4096 and err["tolerance"] == 1e-5
    for s, d in shift.items():
        for p, dp in prec_shift.items():
            e = err["per_solver"][f"{s}/{p}"]
            # the stand-in is rounded to FP32 like the GPU's output
            assert abs(e["max_abs"] - abs(d + dp)) <= 1e-7 and e["rms"] <= e["max_abs"]


def test_measured_issue_and_valu_bound(tmp_path, monkeypatch):
    """The issue-counter summary is read only for the profiled sources, and
    the VALU-bound time prices plain and transcendental instructions at their
    own measured rates."""
    prof = tmp_path / "issue.md"
    monkeypatch.setattr(bench, "ISSUE_PROFILE", str(prof))
    assert bench.measured_issue("offset_sz") is None
    head = ["| bench kernel | waves | VALU / wave | of which trans. F32 | trans. F64 | SALU / wave | x |",
            "|---|---:|---:|---:|---:|---:|---:|",
            "| offset_sz | 262,144 | 493.7 | 33.5 | 0.0 | 221.9 | 1 |"]
    prof.write_text(f"kernel source sha256: `{bench.kernel_source_hash()}`\n\n" + "\n".join(head) + "\n")
    iss = bench.measured_issue("offset_sz")
    assert iss == {"waves": 262144, "valu": 493.7, "trans_f32": 33.5, "trans_f64": 0.0}
    assert bench.measured_issue("volume") is None
    ceiling = {k: {"lane_ops_per_s": 1e12} for k in ("sqrt_f32", "rsq_f32", "rcp_f32", "sin_f32", "exp_f32",
                                                     "log_f32", "rcp_f64", "sqrt_f64")}
    ceiling["sin_f32"] = {"lane_ops_per_s": 0.5e12}                 # the slowest transcendental prices them all
    ceiling["fma_f32"] = {"lane_ops_per_s": 4e12}
    ms = bench.valu_bound_ms(iss, ceiling)
    lanes = 262144 * 64
    assert ms == pytest.approx(1e3 * lanes * ((493.7 - 33.5) / 4e12 + 33.5 / 0.5e12))
    prof.write_text("kernel source sha256: `" + "0" * 64 + "`\n\n" + "\n".join(head) + "\n")
    assert bench.measured_issue("offset_sz") is None


def test_trace_profile_summary(tmp_path):
    """The kernel-trace summary groups dispatches by kernel and launch size,
    with calls and average / minimum duration (ns in the CSV, µs in the
    table), longest total first."""
    head = ('"Kind","Agent_Id","Queue_Id","Stream_Id","Thread_Id","Dispatch_Id","Kernel_Id","Kernel_Name",'
            '"Correlation_Id","Start_Timestamp","End_Timestamp","LDS_Block_Size","Scratch_Size","VGPR_Count",'
            '"Accum_VGPR_Count","SGPR_Count","Workgroup_Size_X","Workgroup_Size_Y","Workgroup_Size_Z",'
            '"Grid_Size_X","Grid_Size_Y","Grid_Size_Z"')
    bwd = '"void plic::(anonymous namespace)::k_offset_bwd<1, float, float, float, 4, true>(float*)"'
    vol = '"void plic::(anonymous namespace)::k_volume<float, float, 4>(float const*, long)"'
    rows = [f'"KERNEL_DISPATCH","Agent 1",1,0,1,{i},1,{bwd},{i},{1000 * i},{1000 * i + d},0,0,64,0,16,512,1,1,'
            f'{g},1,1' for i, (d, g) in enumerate([(435000, 16777216), (425000, 16777216), (100000, 4194304)])]
    rows.append(f'"KERNEL_DISPATCH","Agent 1",1,0,1,9,1,{vol},9,0,230000,0,0,32,0,16,256,1,1,16777216,1,1')
    csvp = tmp_path / "trace.csv"
    csvp.write_text(head + "\n" + "\n".join(rows) + "\n")
    out = bench.write_trace_profile(str(csvp), str(tmp_path / "t.md"))
    text = open(out).read()
    table = [ln for ln in text.splitlines() if ln.startswith("| `")]
    assert table[0].startswith("| `k_offset_bwd<1, float, float, float, 4, true>` | 16,777,216 | 2 | 430.0 | 425.0 |")
    assert table[1].startswith("| `k_volume<float, float, 4>` | 16,777,216 | 1 | 230.0 | 230.0 |")
    assert table[2].startswith("| `k_offset_bwd<1, float, float, float, 4, true>` | 4,194,304 | 1 | 100.0 |")
    assert bench.kernel_source_hash() in text


def test_traffic_profile_lists_the_dispatches_that_ran(tmp_path):
    """A launch is summed over the dispatches that ran: the backward that
    reuses the forward's scan has no scan dispatch, and is listed by the
    others."""
    log2n, n, lat = 10, 1 << 10, 8
    kib = 4 * n / 1024
    items = "void plic::(anonymous namespace)::k_curv_quads<0, float, double, double, true, 0, false>(...)"
    gather = "void plic::(anonymous namespace)::k_curv_gather_direct<false, 0, true>(...)"
    fetch = [("__amd_rocclr_copyBuffer", kib), (items, 1.0), (gather, 2.0)]
    write = [("__amd_rocclr_copyBuffer", kib), (items, 3.0), (gather, 4.0)]
    fc, wc = tmp_path / "fetch.csv", tmp_path / "write.csv"
    write_counters(fc, fetch)
    write_counters(wc, write)
    out = tmp_path / "traffic.md"
    bench.write_traffic_profile(str(fc), str(wc), log2n, lat, str(out))
    rows = {line.split("|")[1].strip(): line for line in out.read_text().splitlines() if line.startswith("| ")}
    cells = [c.strip() for c in rows["curvature_bwd"].split("|")]
    assert "k_curv_scan" not in cells[2] and "k_curv_quads" in cells[2] and "k_curv_gather_direct" in cells[2]
    assert int(cells[3].replace(",", "")) == 1024 * (1 + 2 + 3 + 4)          # copy factors are 1
    assert float(cells[6].replace(",", "")) == 8 * lat ** 3                  # 8 B per cell
