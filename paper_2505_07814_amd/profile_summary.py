"""Summarise rocprofv3 counter runs of bench.py into profiles/*.txt.

FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of a kernel are scaled by the
ratio (known bytes / counted bytes) of a plain device copy of known size
measured in the same run, and written with the hash of the kernel sources
so that bench.py can tell whether they still describe the current kernels.

usage: python -m paper_2505_07814_amd.profile_summary FETCH_CSV WRITE_CSV
           KERNELS OUT_TXT [--launches K] [--grids G1,G2,...] COMMAND...
       python -m paper_2505_07814_amd.profile_summary --activity CSV[,CSV...]
           KERNELS OUT_TXT [--grids G1,G2,...] COMMAND...
       python -m paper_2505_07814_amd.profile_summary --stats STATS_CSV TITLE
           OUT_TXT COMMAND...

KERNELS is a comma-separated list of kernel-name substrings.  Without
--launches the figure is the average per matching dispatch; with it, the
total over all matching dispatches divided by K (for a timed unit made of
several dispatches, such as the N=256 line passes of one gradient).  With
--grids only dispatches of those grid sizes (work-items) count, which keeps
the launches of a timed step apart from other launches of the same kernel in
the profiled run (such as data generation).

--activity summarises SQ / GRBM counter runs (one CSV per pass) of the same
command: each counter's average per matching dispatch, and the busy
fractions rocprofv3 derives per dispatch (over the dispatch's GPU-active
cycles, the largest GRBM_GUI_ACTIVE of the XCDs, and all compute units):
  valu_busy = VALUBusy / 100  (sum of SQ_ACTIVE_INST_VALU / CUs / cycles)
  lds_busy  = LdsUtil / 100   (sum of SQ_LDS_IDX_ACTIVE / CUs / cycles)
  lds_bank_conflict = LDSBankConflict / 100 (sum of SQ_LDS_BANK_CONFLICT / CUs / cycles)
and, where the raw counters were taken, the shares of the resident waves'
cycles spent issuing VALU or waiting for an LDS issue.

--stats turns rocprofv3's kernel statistics (--kernel-trace --stats) into a
table of calls and average / min / max durations per kernel, with the
command and the source hash.
"""
import csv
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# the sources of the multislice forward / gradient kernels and their launches
MULTISLICE_SOURCES = ("constrain.hpp", "kernels.hpp", "lines256.hpp", "ptyr.hip", "wave.hpp")


def source_hash(files=MULTISLICE_SOURCES):
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2505_07814_amd", "csrc")
    for f in sorted(files):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def per_kernel(path, counter, grids=None):
    """{kernel name: [values of counter per dispatch]}; with `grids`, the
    copy kernels and the dispatches of those grid sizes only"""
    out = {}
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        name = r["Kernel_Name"].lower()
        if grids and r.get("Grid_Size") not in grids and "copy" not in name and "elementwise" not in name:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def activity(argv):
    csvs, knames, out_txt = argv[:3]
    rest = argv[3:]
    grids = None
    if rest and rest[0] == "--grids":
        grids = {g for g in rest[1].split(",") if g}
        rest = rest[2:]
    keys = [k for k in knames.split(",") if k]
    vals = {}
    for path in csvs.split(","):
        for r in csv.DictReader(open(path)):
            if not any(q in r["Kernel_Name"] for q in keys):
                continue
            if grids and r.get("Grid_Size") not in grids:
                continue
            vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    avg = {k: sum(v) / len(v) for k, v in sorted(vals.items())}
    lines = [f"# VALU / LDS activity of {knames} (rocprofv3 --pmc, one pass per CSV)",
             f"# command: {' '.join(rest)}"]
    if grids:
        lines.append(f"# dispatches of grid sizes {','.join(sorted(grids, key=int))} only")
    lines.append("# dispatches per counter: " + ", ".join(f"{k} {len(v)}" for k, v in sorted(vals.items())))
    lines += [f"{k} = {v:.6g}" for k, v in avg.items()]
    for derived, key in (("VALUBusy", "valu_busy"), ("LdsUtil", "lds_busy"), ("LDSBankConflict", "lds_bank_conflict")):
        if derived in avg:
            lines.append(f"{key} = {avg[derived] / 100.0:.4f}")
    if "SQ_ACTIVE_INST_VALU" in avg and "SQ_WAVE_CYCLES" in avg:
        lines.append(f"valu_wave_share = {avg['SQ_ACTIVE_INST_VALU'] / avg['SQ_WAVE_CYCLES']:.4f}")
    if "SQ_WAIT_INST_LDS" in avg and "SQ_WAVE_CYCLES" in avg:
        lines.append(f"lds_wait_wave_share = {avg['SQ_WAIT_INST_LDS'] / avg['SQ_WAVE_CYCLES']:.4f}")
    if "SQ_WAIT_ANY" in avg and "SQ_WAVE_CYCLES" in avg:
        lines.append(f"wait_any_wave_share = {avg['SQ_WAIT_ANY'] / avg['SQ_WAVE_CYCLES']:.4f}")
    lines.append(f"source_hash = {source_hash()}")
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def short_name(n):
    n = n.replace("(anonymous namespace)::", "").replace("void ", "")
    if n.startswith("__amd_rocclr"):
        return n.split("(")[0]
    if "at::native" in n or "at::" in n:
        return "torch " + n.split("(")[0].split("::")[-1][:30]
    return n.split("(")[0][:48]


def stats(argv):
    path, title, out_txt = argv[:3]
    cmd = " ".join(argv[3:])
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel statistics, {title}", f"# command: {cmd}",
             f"{'kernel':48s} {'calls':>7s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}"]
    for r in rows:
        lines.append(f"{short_name(r['Name']):48s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.1f} "
                     f"{float(r['MinNs']) / 1e3:10.1f} {float(r['MaxNs']) / 1e3:10.1f} {float(r['Percentage']):6.2f}")
    lines.append(f"source_hash = {source_hash()}")
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines[:12]))


def main(argv):
    if argv and argv[0] == "--activity":
        return activity(argv[1:])
    if argv and argv[0] == "--stats":
        return stats(argv[1:])
    fetch_csv, write_csv, knames, out_txt = argv[:4]
    rest = argv[4:]
    launches = None
    grids = None
    while rest and rest[0] in ("--launches", "--grids"):
        if rest[0] == "--launches":
            launches = int(rest[1])
        else:
            grids = {g for g in rest[1].split(",") if g}
        rest = rest[2:]
    cmd = " ".join(rest)
    keys = [k for k in knames.split(",") if k]
    kname = knames
    fetch = per_kernel(fetch_csv, "FETCH_SIZE", grids)
    write = per_kernel(write_csv, "WRITE_SIZE", grids)
    copy_f = [v for k, v in fetch.items() if "copy" in k.lower() or "elementwise" in k.lower()]
    copy_w = [v for k, v in write.items() if "copy" in k.lower() or "elementwise" in k.lower()]
    big_f = max((x for vals in copy_f for x in vals), default=0.0)
    big_w = max((x for vals in copy_w for x in vals), default=0.0)
    known = 512.0 * 1024                                  # KiB read and written by one copy
    kf = known / big_f if big_f else float("nan")
    kw = known / big_w if big_w else float("nan")
    kf_vals = [v for k, vals in fetch.items() if any(q in k for q in keys) for v in vals]
    kw_vals = [v for k, vals in write.items() if any(q in k for q in keys) for v in vals]
    af = sum(kf_vals) / (launches or len(kf_vals))
    aw = sum(kw_vals) / (launches or len(kw_vals))
    hbm = (af * kf + aw * kw) * 1024
    lines = [
        f"# HBM traffic of {kname} (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)",
        f"# command: {cmd}",
    ] + ([f"# dispatches of grid sizes {','.join(sorted(grids, key=int))} only"] if grids else []) + [
        f"# dispatches: fetch {len(kf_vals)}, write {len(kw_vals)}" + (f", per timed launch of {len(kf_vals) // launches}" if launches else ""),
        f"# copy calibration (512 MiB device copy): FETCH_SIZE {big_f:.0f} KiB, WRITE_SIZE {big_w:.0f} KiB",
        f"fetch_kib_per_launch = {af:.1f}",
        f"write_kib_per_launch = {aw:.1f}",
        f"fetch_scale = {kf:.4f}",
        f"write_scale = {kw:.4f}",
        f"hbm_bytes_per_launch = {hbm:.0f}",
        f"source_hash = {source_hash()}",
    ]
    with open(out_txt, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main(sys.argv[1:])
