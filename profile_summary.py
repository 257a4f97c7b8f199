"""Summarise rocprofv3 output of one bench.py workload into profiles/.

Reads the kernel-trace stats and the FETCH_SIZE / WRITE_SIZE counter passes
produced by

    rocprofv3 --kernel-trace --stats --output-format csv -d DIR -o ks -- CMD
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR -o fetch -- CMD
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR -o write -- CMD

with CMD given on the command line (default: python3 bench.py --workload W
--steps 256 --warmup 16 --no-cpu-baseline --no-tta --calibrate-copy-mb 256), and writes
profiles/kernels_<W>.txt (kernel durations) and profiles/traffic_<W>.txt
(HBM bytes per launch).  Counter values are KiB per dispatch; the plain
256 MiB copy in the same run calibrates them (bytes per counter-KiB).
"""
from __future__ import annotations

import csv
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))


def _rows(path):
    return list(csv.DictReader(open(path)))


# longer names first: "sgep::k_fwd" is a prefix of "sgep::k_fwd2"
_KERNELS = ("k_bpers", "k_bfwd", "k_bcoef", "k_bbwd", "k_wfwd", "k_wmid", "k_wbwd", "k_wprod", "k_wepi",
            "k_winit", "k_fwd2",
            "k_bwdp", "k_fwds", "k_fwd", "k_coefa", "k_coefb", "k_coef", "k_bwd")


def _short(name: str) -> str:
    # the first ICA backward pass is k_bwd with mode argument 4
    if "k_bwd<" in name and "k_bwdp" not in name:
        args = [x.strip() for x in name.split("<", 1)[1].split(">", 1)[0].split(",")]
        if len(args) >= 6 and args[5] == "4":
            return "k_bwd1"
    for k in _KERNELS:
        if k + "<" in name or k + "I" in name or name.startswith(k) or ("::" + k) in name:
            return k
    if "copybuffer" in name.lower():
        return "copy"
    return name[:60]


def main(prof_dir: str, workload: str, cmd: str = "", copy_mib: int = 256):
    """cmd: the exact program line that ran under rocprofv3 (recorded in the
    summaries); copy_mib: size of its calibration copy."""
    sys.path.insert(0, ROOT)
    import bench  # noqa: the source hash of the kernels

    if not cmd:
        cmd = (f"python3 bench.py --workload {workload} --steps 256 --warmup 16 "
               f"--no-cpu-baseline --no-tta --calibrate-copy-mb {copy_mib}")
    ks = _rows(os.path.join(prof_dir, "ks_kernel_stats.csv"))
    out = [f"# rocprofv3 kernel statistics, workload {workload} (MI355X)",
           f"# command: rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o ks -- {cmd}",
           "kernel | calls | avg_us | min_us | max_us | share_%"]
    for r in ks:
        out.append(f"{r['Name'][:90]} | {r['Calls']} | {float(r['AverageNs'])/1e3:.3f} | "
                   f"{float(r['MinNs'])/1e3:.3f} | {float(r['MaxNs'])/1e3:.3f} | "
                   f"{float(r['Percentage']):.2f}")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    open(os.path.join(ROOT, "profiles", f"kernels_{workload}.txt"), "w").write("\n".join(out) + "\n")

    if not os.path.exists(os.path.join(prof_dir, "fetch_counter_collection.csv")):
        print("\n".join(out))
        return  # kernel trace only; no counter passes in this directory
    vals = {}
    for tag, ctr in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        for r in _rows(os.path.join(prof_dir, f"{tag}_counter_collection.csv")):
            if r["Counter_Name"] != ctr:
                continue
            vals.setdefault((_short(r["Kernel_Name"]), tag), []).append(
                (int(r["Grid_Size"]), float(r["Counter_Value"])))
    # the calibration copy: the largest-grid copy dispatches
    def copy_kib(tag):
        c = vals.get(("copy", tag), [])
        big = max(g for g, _ in c)
        return statistics.median(v for g, v in c if g == big)
    scale_r = copy_mib * 2 ** 20 / copy_kib("fetch")   # bytes per counter-KiB, reads
    scale_w = copy_mib * 2 ** 20 / copy_kib("write")   # bytes per counter-KiB, writes
    rec = {"workload": workload,
           "copy_calibration": {"mib": copy_mib, "fetch_kib": copy_kib("fetch"),
                                "write_kib": copy_kib("write"), "read_scale": scale_r,
                                "write_scale": scale_w},
           "kernels": {}}
    lines = [f"# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE, workload {workload}",
             f"# commands: rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o fetch -- {cmd}",
             f"#           rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o write -- {cmd}",
             f"# calibration: plain copy of {copy_mib} MiB reads {copy_kib('fetch'):.0f} KiB and writes "
             f"{copy_kib('write'):.0f} KiB by these counters",
             "kernel | dispatches | fetch_KiB(median) | write_KiB(median) | read_bytes | write_bytes"]
    for k in ("k_fwds", "k_fwd", "k_coef", "k_coefa", "k_coefb", "k_bwdp", "k_bwd1", "k_fwd2", "k_bwd",
              "k_wfwd", "k_wmid", "k_wbwd", "k_wprod", "k_wepi", "k_bfwd", "k_bcoef", "k_bbwd",
              "k_bpers"):
        f = [v for _, v in vals.get((k, "fetch"), [])]
        w = [v for _, v in vals.get((k, "write"), [])]
        if not f:
            continue
        fr, wr = statistics.median(f), statistics.median(w)
        rb, wb = fr * scale_r, wr * scale_w
        rec["kernels"][k] = {"read_bytes": round(rb), "write_bytes": round(wb),
                             "fetch_kib": fr, "write_kib": wr, "dispatches": len(f),
                             "source_hash": bench.kernel_source_hash(bench.KERNEL_HEADER[k])}
        lines.append(f"{k} | {len(f)} | {fr:.1f} | {wr:.1f} | {rb:.0f} | {wb:.0f}")
    lines.append("json: " + json.dumps(rec))
    open(os.path.join(ROOT, "profiles", f"traffic_{workload}.txt"), "w").write("\n".join(lines) + "\n")
    print("\n".join(out + lines))


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2], *(sys.argv[3:4]), *(int(a) for a in sys.argv[4:]))
