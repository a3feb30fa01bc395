"""Condenses rocprofv3 output into the short per-kernel summaries kept under
profiles/, and reads them back.

Inputs are the directories of three rocprofv3 runs of the same bench command:
  --kernel-trace --stats             per-kernel durations
  --pmc FETCH_SIZE  (with --copy-calibration)
  --pmc WRITE_SIZE  (with --copy-calibration)
The bench's --copy-calibration run includes one device copy of exactly
1 GiB; what FETCH_SIZE and WRITE_SIZE read for it gives the factor that
turns each counter into bytes.  HBM traffic per launch of a kernel is
(FETCH_SIZE * fetch factor + WRITE_SIZE * write factor), KiB -> bytes,
averaged over the timed launches.

  python -m paper_2202_05012_amd.prof_summary TRACE_DIR FETCH_DIR WRITE_DIR \\
      --workload NAME --command "..." --out DIR
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_BYTES = 1 << 30          # the calibration copy

# the sources each kernel is built from (a summary is valid while they hash
# to the value it records)
KERNEL_SOURCES = {
    "supa_propagate": ["supa_propagate.hip", "supa_device.hpp"],
    "supa_place": ["supa_place.hip", "supa_device.hpp"],
    "scatter_nodes": ["supa_scatter.hip", "supa_device.hpp"],
    "shapes_kernel": ["supa_shapes.hip"],
    "w1_stats": ["supa_shapes.hip"],
    "w1_hist": ["supa_shapes.hip"],
    "grids_kernel": ["supa_grids.hip"],
    "gate_fused_k256_kernel": ["supa_mlp.hip", "supa_mlp.hpp"],
    "gemm_bf16": ["supa_mlp.hip", "supa_mlp.hpp"],
    "mlp_fused_kernel": ["supa_mlp.hip", "supa_mlp.hpp"],
}


def source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_name(full: str) -> str:
    m = re.search(r"(supa_propagate|supa_place|scatter_nodes|scan_tiles|scan_top|scan_apply|shapes_kernel|"
                  r"shapes_clear|w1_stats|w1_hist|w1_colinfo|w1_distance|w1_groups|w1_zero|grids_kernel|"
                  r"gate_fused_k256_kernel|gemm_bf16|gate_tiles_kernel|gate_rows_kernel|features_kernel|mlp_fused_kernel)\b", full)
    return m.group(1) if m else full


def _rows(d: str, suffix: str):
    files = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    newest = max(files, key=os.path.getmtime)      # a reused directory keeps older runs
    with open(newest) as fh:
        return list(csv.DictReader(fh))


def durations(trace_dir: str):
    """Per kernel: durations (ms) of its dispatches, in order."""
    out = {}
    for r in _rows(trace_dir, "kernel_trace.csv"):
        out.setdefault(short_name(r["Kernel_Name"]), []).append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
    return out


def counter(pmc_dir: str, name: str):
    """Per kernel: counter values (KiB) of its dispatches, in order, and the
    value for the 1 GiB calibration copy."""
    out, copy = {}, None
    for r in _rows(pmc_dir, "counter_collection.csv"):
        if r["Counter_Name"] != name:
            continue
        v = float(r["Counter_Value"])
        k = short_name(r["Kernel_Name"])
        if "copyBuffer" in r["Kernel_Name"]:
            if copy is None or v > copy:
                copy = v
            continue
        out.setdefault(k, []).append(v)
    return out, copy


def steady(vals, skip, last=None):
    """Mean over the dispatches after the first `skip` (sizing probe and
    warm-up), or over the last `last` dispatches when given."""
    if last:
        v = vals[-last:]
    else:
        v = vals[skip:] if len(vals) > skip else vals
    return statistics.fmean(v) if v else float("nan")


def summarize(trace_dir, fetch_dir, write_dir, workload, commands, out_dir, skip=2, kernels=None, last=None):
    dur = durations(trace_dir)
    fetch, fcopy = counter(fetch_dir, "FETCH_SIZE")
    write, wcopy = counter(write_dir, "WRITE_SIZE")
    f_scale = COPY_BYTES / 1024.0 / fcopy if fcopy else float("nan")
    w_scale = COPY_BYTES / 1024.0 / wcopy if wcopy else float("nan")
    written = []
    for k in KERNEL_SOURCES:
        if k not in dur or (kernels and k not in kernels):
            continue
        ms = steady(dur[k], skip, last)
        fk = steady(fetch.get(k, []), skip, last)
        wk = steady(write.get(k, []), skip, last)
        sel = dur[k][-last:] if last else (dur[k][skip:] or dur[k])
        traffic = (fk * f_scale + wk * w_scale) * 1024.0
        lines = [
            f"# {k} -- {workload}",
            "",
            "Commands (run from the repository root; `cd /tmp && export TMPDIR=/tmp` first):",
            "",
            *[f"    {c}" for c in commands],
            "",
            f"source_sha256: {source_hash(k)}",
            (f"dispatches_traced: {len(dur[k])} (averaged: the last {last}, the timed calls)" if last else
             f"dispatches_traced: {len(dur[k])} (first {skip} skipped: sizing or checking call, first warm-up)"),
            f"avg_duration_ms: {ms:.4f}",
            f"min_duration_ms: {min(sel):.4f}",
            f"max_duration_ms: {max(sel):.4f}",
            f"fetch_kib_per_dispatch: {fk:.1f}",
            f"write_kib_per_dispatch: {wk:.1f}",
            f"copy_calibration_fetch_kib: {fcopy:.1f} (1 GiB copy; factor {f_scale:.4f})",
            f"copy_calibration_write_kib: {wcopy:.1f} (1 GiB copy; factor {w_scale:.4f})",
            f"traffic_bytes_per_launch: {traffic:.0f}",
            f"traffic_GBps_at_avg_duration: {traffic / (ms / 1e3) / 1e9:.1f}",
            "",
            "All kernels of the traced run (avg ms over dispatches after the first "
            f"{skip}):",
            "",
            "| kernel | dispatches | avg ms |",
            "|---|---|---|",
            *[f"| {n} | {len(v)} | {steady(v, skip):.4f} |" for n, v in sorted(dur.items())],
            "",
        ]
        path = os.path.join(out_dir, f"{k}_{workload}.md")
        with open(path, "w") as fh:
            fh.write("\n".join(lines))
        written.append(path)
    return written


def read_summary(path: str) -> dict:
    """key: value lines of a summary (values as strings)."""
    d = {}
    with open(path) as fh:
        for line in fh:
            m = re.match(r"^([a-z_0-9]+): (\S+)", line)
            if m:
                d[m.group(1)] = m.group(2)
    return d


def traffic_if_current(profiles_dir: str, kernel: str, workload: str):
    """Measured HBM bytes per launch, or None when there is no summary or
    the kernel's sources changed since it was taken."""
    path = os.path.join(profiles_dir, f"{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    d = read_summary(path)
    if d.get("source_sha256") != source_hash(kernel):
        return None
    try:
        return float(d["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# SIMDs of the device (256 compute units x 4), cycles one wave64 VALU
# instruction holds its 16-lane SIMD, and accelerator dies (GRBM_GUI_ACTIVE
# is summed over the 8 XCDs: it reads about 8x the kernel's clock cycles)
N_SIMD = 1024
VALU_CYCLES = 4
N_XCD = 8


def summarize_counters(pmc_dir, kernel, workload, commands, out_dir, skip=2):
    """Per-dispatch averages of the SQ/GRBM counters of one kernel, and its
    VALU issue fraction: SQ_INSTS_VALU * 4 cycles / (1024 SIMDs * cycles of
    the dispatch), the cycles being GRBM_GUI_ACTIVE / 8 (one GRBM per XCD)."""
    vals = {}
    for r in _rows(pmc_dir, "counter_collection.csv"):
        if short_name(r["Kernel_Name"]) != kernel:
            continue
        vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    avg = {k: steady(v, skip) for k, v in sorted(vals.items())}
    lines = [f"# {kernel} -- instruction counters -- {workload}", "",
             "Command (run from the repository root; `cd /tmp && export TMPDIR=/tmp` first):", "",
             *[f"    {c}" for c in commands], "",
             f"source_sha256: {source_hash(kernel)}",
             f"dispatches: {len(next(iter(vals.values()), []))} (first {skip} skipped)", ""]
    lines += [f"{k}: {v:.0f}" for k, v in avg.items()]
    if "SQ_INSTS_VALU" in avg and avg.get("GRBM_GUI_ACTIVE"):
        cycles = avg["GRBM_GUI_ACTIVE"] / N_XCD
        frac = avg["SQ_INSTS_VALU"] * VALU_CYCLES / (N_SIMD * cycles)
        lines += ["", f"kernel_cycles: {cycles:.0f} (GRBM_GUI_ACTIVE / {N_XCD} XCDs)",
                  f"valu_issue_fraction: {frac:.3f} (SQ_INSTS_VALU * {VALU_CYCLES} / ({N_SIMD} SIMDs * kernel_cycles))"]
        if "SQ_ACTIVE_INST_VALU" in avg:
            busy = avg["SQ_ACTIVE_INST_VALU"] * VALU_CYCLES / (N_SIMD * cycles)
            lines += [f"valu_busy_fraction: {busy:.3f} (SQ_ACTIVE_INST_VALU * {VALU_CYCLES} / ({N_SIMD} SIMDs * "
                      "kernel_cycles))"]
    path = os.path.join(out_dir, f"{kernel}_counters_{workload}.md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return path


def counter_if_current(profiles_dir: str, kernel: str, workload: str, key: str):
    """A value of the kernel's counter summary, or None when there is none or
    the kernel's sources changed since it was taken."""
    path = os.path.join(profiles_dir, f"{kernel}_counters_{workload}.md")
    if not os.path.exists(path):
        return None
    d = read_summary(path)
    if d.get("source_sha256") != source_hash(kernel):
        return None
    try:
        return float(d[key])
    except (KeyError, ValueError):
        return None


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "counters":
        ap = argparse.ArgumentParser()
        ap.add_argument("mode")
        ap.add_argument("pmc_dir")
        ap.add_argument("--kernel", required=True)
        ap.add_argument("--workload", required=True)
        ap.add_argument("--command", action="append", default=[])
        ap.add_argument("--out", required=True)
        ap.add_argument("--skip", type=int, default=2)
        a = ap.parse_args()
        os.makedirs(a.out, exist_ok=True)
        print(summarize_counters(a.pmc_dir, a.kernel, a.workload, a.command, a.out, a.skip))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("trace_dir")
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--out", required=True)
    ap.add_argument("--skip", type=int, default=2)
    ap.add_argument("--kernel", action="append", default=[],
                    help="summarise only these kernels (default: every known kernel traced)")
    ap.add_argument("--last", type=int, default=None,
                    help="average each kernel's last N dispatches (the timed calls) instead")
    a = ap.parse_args()
    os.makedirs(a.out, exist_ok=True)
    for p in summarize(a.trace_dir, a.fetch_dir, a.write_dir, a.workload, a.command, a.out, a.skip,
                       a.kernel or None, a.last):
        print(p)


if __name__ == "__main__":
    main()
