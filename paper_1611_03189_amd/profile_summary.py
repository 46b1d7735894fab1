"""Condense rocprofv3 output into the short text summaries kept beside the measurements.

    python -m paper_1611_03189_amd.profile_summary STATS_CSV "COMMAND" [TITLE] > summary.txt
        one line per kernel with calls, total and mean time (``*_kernel_stats.csv``)
    python -m paper_1611_03189_amd.profile_summary --pmc FETCH_CSV WRITE_CSV CALIB_KERNEL BYTES "COMMANDS"
        per-kernel HBM bytes per dispatch from FETCH_SIZE / WRITE_SIZE counter runs, scaled by
        a copy of known size; prints JSON with the source hashes of the kernels
    python -m paper_1611_03189_amd.profile_summary --mfma COUNTER_CSV "COMMAND" [TITLE]
        per-kernel FP64 matrix-core work from one counter run (SQ_INSTS_VALU_MFMA_MOPS_F64,
        SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE): flops, rate over the dispatches' own
        durations and the fraction of the FP64 matrix peak
"""
import csv
import sys


def summarize(path: str, command: str, title: str = "") -> str:
    rows = list(csv.DictReader(open(path)))
    out = []
    if title:
        out.append(f"# {title}")
    out.append(f"# command: {command}")
    out.append(f"# {'kernel':58s} {'calls':>6s} {'total_ms':>10s} {'mean_us':>10s} {'pct':>6s}")
    for r in rows:
        name = r["Name"]
        if "(" in name:
            name = name[:name.index("(")]
        name = name.replace("void ", "")
        out.append(f"  {name[:58]:58s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e6:10.2f} "
                   f"{float(r['AverageNs']) / 1e3:10.1f} {float(r['Percentage']):6.2f}")
    return "\n".join(out) + "\n"


def pmc_summary(fetch_csv: str, write_csv: str, calib_kernel: str, calib_bytes: float) -> dict:
    """Per-kernel mean FETCH_SIZE and WRITE_SIZE per dispatch (KiB, as the counters report
    them) from two rocprofv3 --pmc runs, and HBM bytes per dispatch after scaling each
    counter by what it reads for a plain copy of known size (calib_bytes read and written)."""
    def per_kernel(path, counter):
        acc = {}
        for r in csv.DictReader(open(path)):
            if r.get("Counter_Name") != counter:
                continue
            name = r["Kernel_Name"]
            if "(" in name:
                name = name[:name.index("(")]
            name = name.replace("void ", "").replace("hs::", "")
            v = acc.setdefault(name, [0.0, 0])
            v[0] += float(r["Counter_Value"])
            v[1] += 1
        return {k: v[0] / v[1] for k, v in acc.items()}

    f = per_kernel(fetch_csv, "FETCH_SIZE")
    w = per_kernel(write_csv, "WRITE_SIZE")
    cal = [k for k in f if calib_kernel in k]
    if not cal:
        raise SystemExit(f"calibration kernel '{calib_kernel}' not found")
    # the copy runs once: its counters over its known traffic give the scale
    f_scale = calib_bytes / (f[cal[0]] * 1024.0)
    w_scale = calib_bytes / (w[cal[0]] * 1024.0)
    out = {"calibration": {"kernel": cal[0], "bytes": calib_bytes, "fetch_kib": f[cal[0]],
                           "write_kib": w[cal[0]], "fetch_scale": f_scale, "write_scale": w_scale},
           "kernels": {}}
    for k in sorted(set(f) | set(w)):
        fb = f.get(k, 0.0) * 1024.0 * f_scale
        wb = w.get(k, 0.0) * 1024.0 * w_scale
        out["kernels"][k] = {"fetch_kib": f.get(k), "write_kib": w.get(k), "hbm_bytes": fb + wb}
    return out


PEAK_FP64_TFLOPS = 78.6          # MI355X dense FP64 (matrix and vector)


def mfma_summary(path: str, command: str, title: str = "") -> str:
    """One line per kernel that issues FP64 MFMA: dispatches, summed dispatch time of the
    counter run, MFMA flops (MOPS_F64 x 512, padding included), their rate over that time, the
    fraction of the FP64 peak, and the MFMA busy cycles over the GUI-active cycles as the
    counters report them (busy summed over the chip's 1024 SIMDs, GUI-active over its 8
    XCDs), and that ratio over 128 SIMDs per XCD: the matrix cores' busy fraction, which the
    flop-based fraction should match."""
    per = {}
    for r in csv.DictReader(open(path)):
        d = per.setdefault(r["Dispatch_Id"], {"name": r["Kernel_Name"],
                                              "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
        d[r["Counter_Name"]] = float(r["Counter_Value"])
    acc = {}
    for d in per.values():
        name = d["name"]
        if "(" in name:
            name = name[:name.index("(")]
        name = name.replace("void ", "")
        a = acc.setdefault(name, [0, 0.0, 0.0, 0.0, 0.0])
        a[0] += 1
        a[1] += d["ns"]
        a[2] += d.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512.0
        a[3] += d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        a[4] += d.get("GRBM_GUI_ACTIVE", 0.0)
    out = []
    if title:
        out.append(f"# {title}")
    out.append(f"# command: {command}")
    out.append(f"# {'kernel':50s} {'calls':>6s} {'ms':>9s} {'mfma_gflop':>11s} {'tflop/s':>8s} "
               f"{'frac':>7s} {'busy/gui':>9s} {'simd_busy':>9s}")
    for name, a in sorted(acc.items(), key=lambda kv: -kv[1][2]):
        if a[2] <= 0.0:
            continue
        rate = a[2] / a[1] / 1e3
        out.append(f"  {name[:50]:50s} {a[0]:6d} {a[1] / 1e6:9.2f} {a[2] / 1e9:11.2f} {rate:8.2f} "
                   f"{rate / PEAK_FP64_TFLOPS:7.4f} {a[3] / max(a[4], 1.0):9.3f} {a[3] / max(a[4], 1.0) / 128:9.4f}")
    return "\n".join(out) + "\n"


def source_hashes() -> dict:
    """sha256 of every HIP source of the library: counters are valid for this code only."""
    import hashlib
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    return {f: hashlib.sha256(open(os.path.join(here, f), "rb").read()).hexdigest()[:16]
            for f in sorted(os.listdir(here)) if f.endswith((".hip", ".h"))}


if __name__ == "__main__":
    if sys.argv[1] == "--mfma":
        print(mfma_summary(sys.argv[2], sys.argv[3], sys.argv[4] if len(sys.argv) > 4 else ""), end="")
    elif sys.argv[1] == "--pmc":
        import json
        res = pmc_summary(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]))
        res["command"] = sys.argv[6]
        res["sources"] = source_hashes()
        print(json.dumps(res, indent=1))
    else:
        print(summarize(sys.argv[1], sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else ""), end="")
