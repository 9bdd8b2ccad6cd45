"""Summaries of rocprofv3 output for the stage kernels.

``python -m paper_2404_08952_amd.profiling <stats_dir> <fetch_dir> <write_dir> <out.md> [--launch-bytes B]``
(``... --mfma <stats_dir> <pmc_dir> <rows>`` instead summarises the indicator
network kernels' matrix-core use from an ``SQ_INSTS_VALU_MFMA_MOPS_BF16`` run)
reads the CSV files that ``rocprofv3 --kernel-trace --stats`` and two
``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of ``bench.py``
wrote, and prints (or writes) a short text summary:

* per-kernel call counts and average durations;
* HBM traffic of the dominant kernel per launch: the FETCH_SIZE and
  WRITE_SIZE counters (KiB per dispatch) scaled by what the same counters
  read for a plain streaming kernel of known size (``bench.py`` runs one:
  ``y = -x`` over 2 GiB of float32), so the factors absorb whatever the
  counters do not see;
* the SHA-256 of the kernel sources the numbers belong to.  ``bench.py``
  reports the traffic only while the sources still hash to that value.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import os
import re
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# sources that the FP32 flux kernel is compiled from
FLUX_SOURCES = ("csrc/residual_impl.hpp", "csrc/dispatch_impl.hpp", "csrc/kernels_f32.hip")
FLUX_KERNEL = r"k_flux<float, 3, 3, 5, true>"
CALIB_KERNEL = r"neg_kernel"
CALIB_BYTES = 2 * 4 * (1 << 29)  # read + write of 2 GiB each


def source_hash(files=FLUX_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _csv(d, pattern):
    files = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not files:
        raise FileNotFoundError(f"no {pattern} under {d}")
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


def kernel_stats(stats_dir):
    rows = _csv(stats_dir, "*kernel_stats.csv")
    out = []
    for r in rows:
        out.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    return sorted(out, key=lambda x: -x[3])


def counter_values(pmc_dir, counter, kernel_regex, largest_grid=False):
    """Counter values of the matching dispatches (with largest_grid, only
    those of the largest grid: the full-size mesh when smaller runs of the
    same kernel share the file)."""
    rows = _csv(pmc_dir, "*counter_collection.csv")
    rx = re.compile(kernel_regex)
    sel = [(int(r["Grid_Size"]), float(r["Counter_Value"])) for r in rows
           if r["Counter_Name"] == counter and rx.search(r["Kernel_Name"])]
    if largest_grid and sel:
        g = max(x[0] for x in sel)
        sel = [x for x in sel if x[0] == g]
    return [v for _g, v in sel]


def traffic(fetch_dir, write_dir, kernel_regex=re.escape(FLUX_KERNEL), calib_regex=CALIB_KERNEL):
    """HBM bytes per launch of the kernel, calibrated on the streaming kernel."""
    f_k = counter_values(fetch_dir, "FETCH_SIZE", kernel_regex, largest_grid=True)
    w_k = counter_values(write_dir, "WRITE_SIZE", kernel_regex, largest_grid=True)
    f_c = counter_values(fetch_dir, "FETCH_SIZE", calib_regex)
    w_c = counter_values(write_dir, "WRITE_SIZE", calib_regex)
    if not (f_k and w_k and f_c and w_c):
        raise ValueError("kernel or calibration dispatches missing from the counter files")
    half = CALIB_BYTES / 2
    ff = half / (statistics.median(f_c) * 1024.0)
    fw = half / (statistics.median(w_c) * 1024.0)
    fetch = statistics.median(f_k) * 1024.0 * ff
    write = statistics.median(w_k) * 1024.0 * fw
    return dict(fetch_bytes=fetch, write_bytes=write, bytes=fetch + write, fetch_factor=ff, write_factor=fw,
                fetch_kib_raw=statistics.median(f_k), write_kib_raw=statistics.median(w_k),
                launches=(len(f_k), len(w_k)))


def read_summary(path):
    """(traffic bytes per launch, source hash) from a summary file, or None."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            m = re.match(r"\s*(traffic_bytes_per_launch|kernel_source_sha256)\s*=\s*(\S+)", line)
            if m:
                vals[m.group(1)] = m.group(2)
    if len(vals) != 2:
        return None
    return float(vals["traffic_bytes_per_launch"]), vals["kernel_source_sha256"]


MFMA_KERNELS = (("k_mlp_fwd", 2 * (24 * 64 + 64 * 64 + 64)), ("k_mlp_grad", 3 * 2 * (24 * 64 + 64 * 64 + 64)))
BF16_PEAK_FLOPS = 2.5e15  # dense matrix-core BF16 peak of the MI355X


def mfma_summary(stats_dir, pmc_dir, rows):
    """Matrix-core use of the indicator network kernels: executed BF16 FLOP
    per launch from SQ_INSTS_VALU_MFMA_MOPS_BF16 (x 512), the rocprofv3
    average duration, and the fraction of the dense BF16 peak; beside it the
    algorithmic FLOP (forward 24 -> 64 -> 64 -> 1 per row, training 3x)."""
    avg = {}
    for name, calls, us, _pct in kernel_stats(stats_dir):
        m = re.search(r"(k_mlp_\w+)", name)
        if m:
            avg[m.group(1)] = (us, calls)
    lines = [f"{'kernel':12s} {'calls':>6s} {'avg_us':>9s} {'MFMA FLOP':>11s} {'TFLOP/s':>8s} {'of peak':>8s}"
             f" {'alg FLOP':>11s}"]
    for k, per_row in MFMA_KERNELS:
        mops = counter_values(pmc_dir, "SQ_INSTS_VALU_MFMA_MOPS_BF16", k)
        flop = statistics.median(mops) * 512.0
        us, calls = avg[k]
        tf = flop / (us * 1e-6) / 1e12
        lines.append(f"{k:12s} {calls:6d} {us:9.1f} {flop:11.4e} {tf:8.1f} {tf * 1e12 / BF16_PEAK_FLOPS:8.4f}"
                     f" {per_row * rows:11.4e}")
    return lines


def main(argv):
    if len(argv) >= 2 and argv[1] == "--mfma":
        if len(argv) < 5:
            print(__doc__)
            return 2
        lines = mfma_summary(argv[2], argv[3], int(argv[4]))
        print("\n".join(lines))
        return 0
    if len(argv) < 5:
        print(__doc__)
        return 2
    stats_dir, fetch_dir, write_dir, out = argv[1:5]
    launch_bytes = None
    if "--launch-bytes" in argv:
        launch_bytes = float(argv[argv.index("--launch-bytes") + 1])
    lines = []
    lines.append("kernel statistics (rocprofv3 --kernel-trace --stats):")
    lines.append(f"{'kernel':80s} {'calls':>6s} {'avg_us':>10s} {'pct':>7s}")
    for name, calls, avg, pct in kernel_stats(stats_dir)[:14]:
        lines.append(f"{name[:80]:80s} {calls:6d} {avg:10.1f} {pct:7.2f}")
    t = traffic(fetch_dir, write_dir)
    lines.append("")
    lines.append(f"HBM traffic of {FLUX_KERNEL} per launch (median over {t['launches'][0]} dispatches):")
    lines.append(f"  FETCH_SIZE {t['fetch_kib_raw']:.0f} KiB x {t['fetch_factor']:.3f} = {t['fetch_bytes'] / 1e9:.3f} GB")
    lines.append(f"  WRITE_SIZE {t['write_kib_raw']:.0f} KiB x {t['write_factor']:.3f} = {t['write_bytes'] / 1e9:.3f} GB")
    lines.append("  (factors: the same counters on the 2 GiB streaming kernel y = -x, whose true traffic is"
                 " 2 GiB read + 2 GiB written)")
    if launch_bytes:
        lines.append(f"  algorithmic bytes per launch {launch_bytes / 1e9:.3f} GB; measured / algorithmic = "
                     f"{t['bytes'] / launch_bytes:.2f}")
    lines.append(f"traffic_bytes_per_launch = {t['bytes']:.6e}")
    lines.append(f"kernel_source_sha256 = {source_hash()}")
    text = "\n".join(lines) + "\n"
    if out == "-":
        print(text)
    else:
        with open(out, "a") as fh:
            fh.write(text)
        print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
