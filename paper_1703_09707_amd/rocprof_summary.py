"""Short text summaries of rocprofv3 runs (rocpd SQLite databases).

    python -m paper_1703_09707_amd.rocprof_summary --kernel shoot_fp64_kernel \\
        --stats prof_stats/bench_results.db \\
        --fetch prof_fetch/bench_results.db \\
        --write prof_write/bench_results.db \\
        --valu prof_valu/bench_results.db \\
        --copy-mib 1024 --command "..." --out profiles/<kernel>_<workload>.txt

HBM byte counters are scaled by what the same counter reads for a plain copy
of a known size (bench.py --copy-calibration MIB copies MIB MiB three times):
scale = expected KiB / measured KiB.  The summary records a SHA-256 of the
kernel's sources so that a later change of the kernel invalidates it.
"""
import argparse
import hashlib
import os
import sqlite3

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = {
    "shoot_fp64_kernel": ["csrc/shoot_fp64.hip", "csrc/ray_common.h", "csrc/raysh_internal.h"],
    "shoot_fp32_kernel": ["csrc/shoot_fp32.hip", "csrc/ray_common.h", "csrc/raysh_internal.h"],
    "batch_fp64_kernel": ["csrc/shoot_fp64.hip", "csrc/ray_common.h", "csrc/raysh_internal.h"],
    "batch_fp32_kernel": ["csrc/shoot_fp32.hip", "csrc/ray_common.h", "csrc/raysh_internal.h"],
    "partial_fp64_kernel": ["csrc/shoot_fp64.hip", "csrc/ray_common.h", "csrc/raysh_internal.h"],
    "finish_fp64_kernel": ["csrc/shoot_fp64.hip", "csrc/ray_common.h", "csrc/raysh_internal.h"],
    "expansion_fp64_kernel": ["csrc/shoot_expansion.hip", "csrc/ray_common.h", "csrc/raysh_internal.h"],
    "expansion_block_kernel": ["csrc/shoot_expansion.hip", "csrc/ray_common.h", "csrc/raysh_internal.h"],
    "light_curve_kernel": ["csrc/light_curves.hip", "csrc/smooth.h"],
    "light_curve_track_kernel": ["csrc/light_curves.hip", "csrc/smooth.h"],
}


def source_hash(kernel):
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _rows(db, sql, args=()):
    con = sqlite3.connect(db)
    try:
        return con.execute(sql, args).fetchall()
    finally:
        con.close()


def kernel_stats(db):
    return _rows(db, "select name, total_calls, total_duration, average, percentage from top_kernels")


def counter_values(db, name_like, grid=None):
    """{counter: [total per dispatch]} for kernels whose name contains
    name_like, optionally only dispatches of one grid size (threads).  The
    totals are rocprofv3's per-dispatch values, summed over the hardware
    instances of each counter."""
    out = {}
    sql = "select counter_name, value, grid_size from counters_collection where kernel_name like ?"
    for counter, value, g in _rows(db, sql, (f"%{name_like}%",)):
        if grid is None or g == grid:
            out.setdefault(counter, []).append(value)
    return out


def dispatch_durations_us(db, name_like, grid=None):
    """Durations (us) of the kernel's dispatches, optionally only those of
    one grid size (threads)."""
    sql = "select duration, grid_x * grid_y * grid_z from kernels where name like ?"
    out = []
    for dur, g in _rows(db, sql, (f"%{name_like}%",)):
        if grid is None or g == grid:
            out.append(dur / 1000.0)
    return out


def per_instance_mean(db, name_like, counter, grid=None):
    """Mean over hardware instances and dispatches of one counter (for
    counters kept per XCD, such as GRBM_GUI_ACTIVE, whose instance mean is
    the dispatch's length in cycles)."""
    ids = {d for d, g in _rows(db, "select dispatch_id, grid_size from counters_collection "
                                   "where kernel_name like ? and counter_name = ?", (f"%{name_like}%", counter))
           if grid is None or g == grid}
    vals = [v for d, v in _rows(db, "select dispatch_id, counter_value from pmc_events "
                                    "where name like ? and counter_name = ?", (f"%{name_like}%", counter))
            if d in ids]
    return sum(vals) / len(vals) if vals else None


def dispatch_waves(db, name_like, grid=None):
    """Waves of one dispatch of the kernel (grid size / 64)."""
    for (g,) in _rows(db, "select grid_size from counters_collection where kernel_name like ?", (f"%{name_like}%",)):
        if grid is None or g == grid:
            return g / 64.0
    return None


def pmc_lines(dbs, kernel, grid, n_cu):
    """Every counter of the kernel's dispatches in the given databases (mean
    per dispatch, summed over hardware instances), and for counters of
    cycles (busy, stall) their share of the CUs' cycles: value / (n_cu x the
    dispatch's GRBM_GUI_ACTIVE per XCD)."""
    vals, cycles = {}, None
    for db in dbs:
        for k, v in counter_values(db, kernel, grid).items():
            vals[k] = sum(v) / len(v)
        g = per_instance_mean(db, kernel, "GRBM_GUI_ACTIVE", grid)
        if g:
            cycles = g
    out = ["memory-pipeline counters per dispatch (sum over instances):"]
    for k in sorted(vals):
        line = f"  {k}: {vals[k]:.4e}"
        if cycles and k != "GRBM_GUI_ACTIVE" and ("BUSY" in k or "STALL" in k):
            line += f"  ({vals[k] / (n_cu * cycles):.3f} of {n_cu} CUs' cycles)"
        out.append(line)
    if cycles:
        out.append(f"cycles_per_dispatch: {cycles:.4e}  (GRBM_GUI_ACTIVE per XCD)")
    return out


def probe_lines(valu_db, stats_db, precision, expected_fma):
    """The FMA probe (raysh_fma_probe) profiled in the same run: its FMA
    counter per dispatch against the wave-level FMA instructions it is known
    to issue, and the FLOP rate the counters then give over its time."""
    P = precision.upper()
    name = "fma_probe_kernel<double>" if precision == "f64" else "fma_probe_kernel<float>"
    vals = counter_values(valu_db, name)
    fma = vals.get(f"SQ_INSTS_VALU_FMA_{P}")
    out = [f"FMA probe ({name}, the counters' calibration):"]
    if not fma:
        return out + ["  not in this run"]
    counted = sum(fma) / len(fma)
    out.append(f"  SQ_INSTS_VALU_FMA_{P} per dispatch: {counted:.6e}  (known: {expected_fma:.6e} wave "
               f"instructions; ratio {counted / expected_fma:.4f})")
    durs = dispatch_durations_us(stats_db, name) or dispatch_durations_us(valu_db, name)
    if durs:
        us = sorted(durs)[len(durs) // 2]
        tflops = 64 * 2 * counted / (us * 1e-6) / 1e12
        out.append(f"  median duration {us:.1f} us: 64 lanes x 2 FLOP x the counter = {tflops:.2f} TFLOP/s "
                   f"({tflops / 78.6:.3f} of 78.6)")
    return out


def read_summary(path):
    """key: value pairs of a summary file (None if missing)."""
    if not os.path.exists(path):
        return None
    out = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--valu")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--command", default="")
    ap.add_argument("--workload", default="")
    ap.add_argument("--flop-per-launch", type=float, default=None)
    ap.add_argument("--precision", choices=("f64", "f32"), default="f64",
                    help="the VALU precision of the kernel's FLOP counters")
    ap.add_argument("--grid", type=int, default=None,
                    help="only dispatches of this grid size (threads) give the kernel's time")
    ap.add_argument("--pmc", nargs="*", default=[],
                    help="more --pmc databases: every counter of the kernel is listed, and those counted in "
                         "cycles also as a fraction of the CUs' cycles (GRBM_GUI_ACTIVE in one of them)")
    ap.add_argument("--n-cu", type=int, default=256)
    ap.add_argument("--probe-fma", type=float, default=None,
                    help="wave-level FMA instructions per dispatch of the FMA probe in the --valu run: "
                         "the summary checks the counter against it")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)

    lines = [f"kernel: {a.kernel}", f"workload: {a.workload}", f"source_sha256: {source_hash(a.kernel)}",
             f"command: {a.command}", ""]
    lines.append("kernel trace (rocprofv3 --kernel-trace --stats), durations in us:")
    k_avg = None
    for name, calls, total, avg, pct in kernel_stats(a.stats)[:8]:
        short = name.replace("(anonymous namespace)::", "").split("(")[0][-70:]
        lines.append(f"  {short:70s} calls {calls:4d} avg {avg:14.1f} total {total:16.1f} {pct:6.2f}%")
        if a.kernel in name and k_avg is None:
            k_avg = avg
    lines.append("")
    durs = dispatch_durations_us(a.stats, a.kernel, a.grid)
    if durs:
        k_avg = sum(durs) / len(durs)
        lines.append(f"dispatches: {len(durs)}" + (f" (grid {a.grid} threads)" if a.grid else ""))
    lines.append(f"avg_us: {k_avg}")
    expected_kib = a.copy_mib * 1024.0
    traffic = 0.0
    have = 0
    for label, db, counter in (("fetch", a.fetch, "FETCH_SIZE"), ("write", a.write, "WRITE_SIZE")):
        if not db:
            continue
        copy = counter_values(db, "copyBuffer").get(counter) or counter_values(db, "copy").get(counter)
        kern = counter_values(db, a.kernel, a.grid).get(counter)
        if not copy or not kern:
            continue
        c = sum(copy) / len(copy)
        k = sum(kern) / len(kern)
        scale = expected_kib / c
        lines.append(f"{label}_copy_kib_per_dispatch: {c:.1f}  (copy of {a.copy_mib} MiB: expected {expected_kib:.0f})")
        lines.append(f"{label}_scale: {scale:.4f}")
        lines.append(f"{label}_kib_per_dispatch: {k:.1f}")
        lines.append(f"{label}_bytes_per_launch: {k * scale * 1024:.0f}")
        traffic += k * scale * 1024
        have += 1
    if have == 2:
        lines.append(f"traffic_bytes_per_launch: {traffic:.0f}")
    if a.valu:
        vals = counter_values(a.valu, a.kernel, a.grid)
        if vals:
            lines.append("")
            avg = {k: sum(v) / len(v) for k, v in vals.items()}
            waves = dispatch_waves(a.valu, a.kernel, a.grid)
            # a check that the SQ counters saw every wave of the dispatch (1.0);
            # were it below one, they would be scaled by it
            factor = waves / avg["SQ_WAVES"] if waves and avg.get("SQ_WAVES") else 1.0
            lines.append(f"dispatch_waves: {waves}")
            lines.append(f"sq_sample_factor: {factor:.3f}  (dispatch waves / SQ_WAVES)")
            lines.append("VALU counters per dispatch (wave instructions; then x sq_sample_factor):")
            for k in sorted(avg):
                scaled = avg[k] * factor if k.startswith("SQ_") else avg[k]
                lines.append(f"  {k}: {avg[k]:.6e}  ->  {scaled:.6e}")
            avg = {k: (v * factor if k.startswith("SQ_") else v) for k, v in avg.items()}
            P = a.precision.upper()
            f64 = 64 * (avg.get(f"SQ_INSTS_VALU_ADD_{P}", 0) + avg.get(f"SQ_INSTS_VALU_MUL_{P}", 0) +
                        avg.get(f"SQ_INSTS_VALU_TRANS_{P}", 0) + 2 * avg.get(f"SQ_INSTS_VALU_FMA_{P}", 0))
            tag = "fp64" if a.precision == "f64" else "fp32"
            lines.append(f"counter_flop_{tag}_per_launch: {f64:.6e}")
            if k_avg:
                sec = k_avg * 1e-6
                lines.append(f"counter_tflops_{tag}: {f64 / sec / 1e12:.3f}")
                grbm = per_instance_mean(a.valu, a.kernel, "GRBM_GUI_ACTIVE", a.grid)
                if grbm:
                    clock = grbm / sec
                    lines.append(f"mean_clock_ghz: {clock / 1e9:.3f}  (GRBM_GUI_ACTIVE per XCD / kernel time)")
                if "SQ_INSTS_VALU" in avg and waves:
                    simds = 1024   # 256 CUs x 4 SIMDs
                    busy = avg["SQ_INSTS_VALU"] * 4 / simds / sec
                    lines.append(f"valu_issue_cycles_per_second_per_simd: {busy:.4e}  "
                                 "(a wave64 VALU instruction takes 4 cycles of a 16-lane SIMD)")
                    if grbm:
                        lines.append(f"valu_issue_fraction: {busy / clock:.3f}  (of the measured clock)")
            if a.flop_per_launch:
                lines.append(f"algorithmic_flop_per_launch: {a.flop_per_launch:.6e}")
                lines.append(f"counter_over_algorithmic: {f64 / a.flop_per_launch:.4f}")
    if a.valu and a.probe_fma:
        lines += [""] + probe_lines(a.valu, a.stats, a.precision, a.probe_fma)
    if a.pmc:
        lines += [""] + pmc_lines(a.pmc, a.kernel, a.grid, a.n_cu)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
