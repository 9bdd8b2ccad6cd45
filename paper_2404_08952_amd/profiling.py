"""Summaries of rocprofv3 output for the stage kernels.

``python -m paper_2404_08952_amd.profiling <stats_dir> <fetch_dir> <write_dir> <out.md> ["<kernel>=<bytes>" ...]``
(``... --mfma <stats_dir> <pmc_dir> <rows>`` instead summarises the indicator
network kernels' matrix-core use from an ``SQ_INSTS_VALU_MFMA_MOPS_BF16`` run;
``... --busy <sq_dir> <ta_dir>`` the stage kernels' vector-issue
and texture-address shares from two counter runs, see ``busy_summary``)
reads the CSV files that ``rocprofv3 --kernel-trace --stats`` and two
``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of ``bench.py``
wrote, and prints (or writes) a short text summary:

* per-kernel call counts and average durations;
* HBM traffic per launch of every stage kernel: the FETCH_SIZE and
  WRITE_SIZE counters (KiB per dispatch) scaled by what the same counters
  read for a plain streaming kernel of known size (``bench.py`` runs one:
  ``y = -x`` over 2 GiB of float32), so the factors absorb whatever the
  counters do not see; beside it the algorithmic bytes given on the command
  line (``bench.py`` prints them);
* the SHA-256 of the kernel sources the numbers belong to (their code with
  comments stripped).  ``bench.py`` reports the traffic only while the
  sources still hash to that value.
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
# sources that the stage kernels are compiled from
FLUX_SOURCES = ("csrc/residual_impl.hpp", "csrc/dispatch_impl.hpp", "csrc/kernels_f32.hip",
                "csrc/indicator_impl.hpp", "csrc/indicator.hip", "csrc/coefficients.hpp")
FLUX_KERNEL = r"k_flux<float, 3, 3, 5, true, 2, 0(, \d+)?>"
# the stage kernels of the headline workload (USR5 + HLLC + learned blend):
# short name -> kernel-name pattern, FP32 (cell-reference form) and FP64
STAGE_KERNELS = (
    ("fp32 k_flux", FLUX_KERNEL),
    ("fp32 k_grad_features", re.escape("k_grad_features<float, 3>")),
    ("fp32 k_hface", re.escape("k_hface_w5<float, 3, 5>")),
    ("fp64 k_flux", r"k_flux<double, 3, 3, 5, true, 0, 0(, \d+)?>"),
    ("fp64 k_grad_features", re.escape("k_grad_features<double, 3>")),
    ("fp64 k_hface", re.escape("k_hface<double, 3, 5>")),
    ("k_mlp_fwd", re.escape("k_mlp_fwd")),
)
CALIB_KERNEL = r"neg_kernel"
CALIB_BYTES = 2 * 4 * (1 << 29)  # read + write of 2 GiB each


def _code_only(text: str) -> str:
    """The source without comments and with whitespace collapsed: edits to
    comments leave the compiled kernels, and so the hash, unchanged."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_hash(files=FLUX_SOURCES, read=None) -> str:
    """SHA-256 over the code (comments stripped) of the kernel sources;
    read(path) -> text may supply another version of each file."""
    h = hashlib.sha256()
    for f in files:
        if read is None:
            with open(os.path.join(HERE, f)) as fh:
                text = fh.read()
        else:
            text = read(f)
        h.update(_code_only(text).encode())
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


def traffic(fetch_dir, write_dir, kernel_regex=FLUX_KERNEL, calib_regex=CALIB_KERNEL):
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
    """({short kernel name: traffic bytes per launch}, source hash) from a
    summary file, or None."""
    if not os.path.exists(path):
        return None
    per, sha = {}, None
    with open(path) as fh:
        for line in fh:
            m = re.match(r"\s*traffic_bytes_per_launch\[(.+)\]\s*=\s*(\S+)", line)
            if m:
                per[m.group(1)] = float(m.group(2))
            m = re.match(r"\s*kernel_source_sha256\s*=\s*(\S+)", line)
            if m:
                sha = m.group(1)
    if not per or sha is None:
        return None
    return per, sha


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


# per-SIMD issue cost of one wave64 instruction on a 16-lane SIMD, in cycles
VALU_ISSUE_CYCLES = 4
N_XCC = 8
N_SIMD = 1024  # 256 CUs x 4 SIMDs


def dispatch_us(pmc_dir, counter, kernel_regex):
    """Durations (us) of the matching full-size dispatches of a counter run,
    from their start and end timestamps (ns)."""
    rows = _csv(pmc_dir, "*counter_collection.csv")
    rx = re.compile(kernel_regex)
    sel = [(int(r["Grid_Size"]), (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3) for r in rows
           if r["Counter_Name"] == counter and rx.search(r["Kernel_Name"])]
    if not sel:
        return []
    g = max(x[0] for x in sel)
    return [us for gg, us in sel if gg == g]


def busy_summary(sq_dir, ta_dir):
    """Where the stage kernels spend their cycles, from two counter runs
    (one dispatch at a time, so the network does not share the chip):
    SQ_INSTS_VALU / SQ_INSTS_VALU_TRANS_F32 / SQ_WAVES with GRBM_GUI_ACTIVE,
    and TA_BUSY_avr / TA_ADDR_STALLED_BY_TC_CYCLES_sum with GRBM_GUI_ACTIVE.
    Per kernel (median over its full-size dispatches): the dispatch's
    duration and GPU cycles (GRBM_GUI_ACTIVE summed over the 8 XCDs, so / 8),
    VALU and transcendental instructions per wave, the VALU issue share
    (instructions x 4 cycles over the SIMDs' cycles: a lower bound on the
    vector units' busy time, since transcendentals take longer), and the
    texture-address unit's busy share (TA_BUSY_avr over the cycles)."""
    lines = [f"{'kernel':22s} {'us':>8s} {'GPU cycles':>11s} {'MHz':>6s} {'VALU/wave':>10s} {'trans/wave':>10s}"
             f" {'VALU issue':>10s} {'TA busy':>8s} {'TA addr stalled by TC':>22s}"]
    for short, rx in STAGE_KERNELS:
        gui = counter_values(sq_dir, "GRBM_GUI_ACTIVE", rx, largest_grid=True)
        if not gui:
            continue
        us = statistics.median(dispatch_us(sq_dir, "GRBM_GUI_ACTIVE", rx))
        cyc = statistics.median(gui) / N_XCC
        valu = statistics.median(counter_values(sq_dir, "SQ_INSTS_VALU", rx, largest_grid=True))
        trans = statistics.median(counter_values(sq_dir, "SQ_INSTS_VALU_TRANS_F32", rx, largest_grid=True))
        waves = statistics.median(counter_values(sq_dir, "SQ_WAVES", rx, largest_grid=True))
        gui_ta = statistics.median(counter_values(ta_dir, "GRBM_GUI_ACTIVE", rx, largest_grid=True)) / N_XCC
        ta = statistics.median(counter_values(ta_dir, "TA_BUSY_avr", rx, largest_grid=True))
        stall = statistics.median(counter_values(ta_dir, "TA_ADDR_STALLED_BY_TC_CYCLES_sum", rx, largest_grid=True))
        issue = valu * VALU_ISSUE_CYCLES / (N_SIMD * cyc)
        lines.append(f"{short:22s} {us:8.1f} {cyc:11.4e} {cyc / us:6.0f} {valu / waves:10.1f} {trans / waves:10.1f}"
                     f" {issue:10.3f} {ta / gui_ta:8.3f} {stall:22.4e}")
    return lines


def main(argv):
    if len(argv) >= 2 and argv[1] == "--busy":
        if len(argv) < 4:
            print("usage: python -m paper_2404_08952_amd.profiling --busy <sq_pmc_dir> <ta_pmc_dir>")
            return 2
        print("\n".join(busy_summary(argv[2], argv[3])))
        print(f"kernel_source_sha256 = {source_hash()}")
        return 0
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
    # algorithmic bytes per launch: --bytes "fp32 k_flux=9.0e9" ...
    alg = {}
    for a in argv[5:]:
        if "=" in a:
            k, v = a.rsplit("=", 1)
            alg[k] = float(v)
    stats = kernel_stats(stats_dir)
    lines = []
    lines.append("kernel statistics (rocprofv3 --kernel-trace --stats):")
    lines.append(f"{'kernel':80s} {'calls':>6s} {'avg_us':>10s} {'pct':>7s}")
    for name, calls, avg, pct in stats[:16]:
        lines.append(f"{name[:80]:80s} {calls:6d} {avg:10.1f} {pct:7.2f}")
    lines.append("")
    lines.append("HBM traffic per launch of the stage kernels (FETCH_SIZE and WRITE_SIZE, median over the")
    lines.append("full-size dispatches, calibrated on the 2 GiB streaming kernel y = -x whose true traffic is")
    lines.append("2 GiB read + 2 GiB written), against the kernel's algorithmic bytes:")
    lines.append(f"{'kernel':22s} {'avg_us':>8s} {'fetch GB':>9s} {'write GB':>9s} {'traffic GB':>10s} {'TB/s':>6s}"
                 f" {'alg GB':>8s} {'alg TB/s':>9s} {'traffic/alg':>11s}")
    traffic_lines = []
    for short, rx in STAGE_KERNELS:
        try:
            t = traffic(fetch_dir, write_dir, kernel_regex=rx)
        except ValueError:
            continue
        us = [a for n, _c, a, _p in stats if re.search(rx, n)]
        us = us[0] if us else float("nan")
        ag = alg.get(short)
        lines.append(f"{short:22s} {us:8.1f} {t['fetch_bytes'] / 1e9:9.3f} {t['write_bytes'] / 1e9:9.3f}"
                     f" {t['bytes'] / 1e9:10.3f} {t['bytes'] / (us * 1e-6) / 1e12:6.2f}"
                     + (f" {ag / 1e9:8.3f} {ag / (us * 1e-6) / 1e12:9.2f} {t['bytes'] / ag:11.2f}" if ag else ""))
        traffic_lines.append(f"traffic_bytes_per_launch[{short}] = {t['bytes']:.6e}")
        if ag:
            traffic_lines.append(f"algorithmic_bytes_per_launch[{short}] = {ag:.6e}")
    t = traffic(fetch_dir, write_dir, kernel_regex=FLUX_KERNEL)
    lines.append(f"  (calibration factors: FETCH_SIZE x {t['fetch_factor']:.3f}, WRITE_SIZE x {t['write_factor']:.3f})")
    lines += traffic_lines
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
