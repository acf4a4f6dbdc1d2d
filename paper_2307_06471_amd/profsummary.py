"""Short text summaries of rocprofv3 output, for the files under profiles/.

  python -m paper_2307_06471_amd.profsummary stats <kernel_stats.csv> <out.txt> <title> <command>
      per-kernel calls, average and total duration (from --kernel-trace --stats)

  python -m paper_2307_06471_amd.profsummary counters <counter_collection.csv>
      "<kernel>;<kernel>;..." <out.txt> <command>
      per-dispatch SQ/GRBM counter averages of the named kernels and the
      VALU-instructions-per-wave, VALU-busy, MFMA-busy and memory-wait ratios

  python -m paper_2307_06471_amd.profsummary traffic <fetch counter_collection.csv>
      <write counter_collection.csv> <kernel substring> <copy_bytes> <out.txt> <command>
      HBM traffic of one kernel per launch: FETCH_SIZE and WRITE_SIZE (KiB per
      dispatch) averaged over its dispatches, each scaled by the ratio of a
      plain device copy's known size to what the same counter reads for it
      (the largest copy dispatch in the same run), plus the hash of the kernel
      sources it was measured on (the benchmark reports the traffic only while
      the sources still hash the same).
"""
import csv
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/crkdg_kernels.hip", "csrc/dg_core.hpp", "csrc/crkdg_internal.hpp",
                  "csrc/mlp_core.hpp")


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stats(path, out, title, command):
    rows = list(csv.DictReader(open(path)))
    lines = [f"# {title}", "", "command (repo root on the MI355X box, after "
             "`cd /tmp && export TMPDIR=/tmp`):", f"  {command}", "",
             f"kernel source hash: {kernel_source_hash()}", "",
             "%-72s %7s %11s %11s %7s" % ("kernel", "calls", "avg_us", "total_ms", "pct")]
    for d in rows:
        n = d["Name"].replace("crk::", "")
        if len(n) > 72:
            n = n[:69] + "..."
        lines.append("%-72s %7s %11.1f %11.3f %7.2f" % (
            n, d["Calls"], float(d["AverageNs"]) / 1e3, float(d["TotalDurationNs"]) / 1e6,
            float(d["Percentage"])))
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def _per_dispatch(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    return rows


def traffic(fetch_csv, write_csv, kernel, copy_bytes, out, command):
    res = {}
    for name, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        rows = _per_dispatch(path, counter)
        names = {r["Kernel_Name"] for r in rows if kernel in r["Kernel_Name"]}
        if len(names) > 1:  # one template instance per summary
            raise SystemExit(f"{kernel!r} matches {len(names)} kernels in {path}")
        kern = [float(r["Counter_Value"]) for r in rows if kernel in r["Kernel_Name"]]
        copies = [r for r in rows if "copy" in r["Kernel_Name"].lower()]
        if not kern or not copies:
            raise SystemExit(f"no {counter} rows for {kernel!r} or for a copy kernel in {path}")
        big = max(int(r["Grid_Size"]) for r in copies)
        cval = [float(r["Counter_Value"]) for r in copies if int(r["Grid_Size"]) == big]
        kib_copy = sum(cval) / len(cval)
        factor = copy_bytes / (kib_copy * 1024.0)
        kib = sum(kern) / len(kern)
        res[name] = {"kib_per_dispatch": kib, "dispatches": len(kern), "copy_kib": kib_copy,
                     "factor": factor, "bytes_per_launch": kib * 1024.0 * factor}
    # WRITE_SIZE counts a copy's written bytes exactly on this hardware: a
    # factor far from 1 means the largest copy is not the calibration copy
    if abs(res["write"]["factor"] - 1.0) > 0.1:
        raise SystemExit(f"calibration copy mismatch: write factor {res['write']['factor']:.3f}")
    lines = [f"# HBM traffic per launch of {kernel}", "",
             "commands (repo root on the MI355X box, after `cd /tmp && export TMPDIR=/tmp`):",
             f"  {command}", "",
             f"kernel source hash: {kernel_source_hash()}",
             f"calibration copy bytes: {int(copy_bytes)}"]
    for name in ("fetch", "write"):
        r = res[name]
        lines += [f"{name}_kib_per_dispatch: {r['kib_per_dispatch']:.1f}",
                  f"{name}_dispatches: {r['dispatches']}",
                  f"{name}_copy_kib: {r['copy_kib']:.1f}",
                  f"{name}_factor: {r['factor']:.5f}",
                  f"{name}_bytes_per_launch: {r['bytes_per_launch']:.0f}"]
    lines.append(f"traffic_bytes_per_launch: {res['fetch']['bytes_per_launch'] + res['write']['bytes_per_launch']:.0f}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


def counters(csv_path, kernels, out, command, simds=1024, xcds=8):
    """per-dispatch averages of the SQ/GRBM counters of one rocprofv3 --pmc
    run for each kernel name given in full, and three ratios:
      valu_insts_per_wave = SQ_INSTS_VALU / SQ_WAVES
      valu_busy = 4 SQ_ACTIVE_INST_VALU / (simds * GRBM_GUI_ACTIVE / xcds)
        (SQ_ACTIVE_INST_VALU counts in units of 4 cycles; GRBM_GUI_ACTIVE is
        summed over the XCDs)
      wait_fraction = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES (share of the waves'
        lifetime spent waiting for memory results)
    and, when counted, mfma_busy = SQ_VALU_MFMA_BUSY_CYCLES / (simds *
    GRBM_GUI_ACTIVE / xcds) and mfma_bf16_flop = 512 SQ_INSTS_VALU_MFMA_MOPS_BF16
    per dispatch; with the SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_{F32,F64} counters,
    the executed vector flops per dispatch (64 lanes per instruction, two
    flops per FMA)"""
    rows = list(csv.DictReader(open(csv_path)))
    lines = [f"# SQ counters per dispatch", "",
             "command (repo root on the MI355X box, after `cd /tmp && export TMPDIR=/tmp`):",
             f"  {command}", "", f"kernel source hash: {kernel_source_hash()}", ""]
    for k in kernels:
        vals = {}
        for r in rows:
            name = r["Kernel_Name"]
            if name.startswith("void "):
                name = name[5:]
            if name.split("(")[0].replace("crk::", "") != k:
                continue
            vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        if not vals:
            raise SystemExit(f"no rows for kernel {k!r} in {csv_path}")
        avg = {c: sum(v) / len(v) for c, v in vals.items()}
        lines.append(f"{k}: dispatches {len(next(iter(vals.values())))}")
        for c in sorted(avg):
            lines.append(f"  {c}: {avg[c]:.6g}")
        if "SQ_INSTS_VALU" in avg and "SQ_WAVES" in avg:
            lines.append(f"  valu_insts_per_wave: {avg['SQ_INSTS_VALU'] / avg['SQ_WAVES']:.1f}")
        if "SQ_ACTIVE_INST_VALU" in avg and "GRBM_GUI_ACTIVE" in avg:
            busy = 4.0 * avg["SQ_ACTIVE_INST_VALU"] / (simds * avg["GRBM_GUI_ACTIVE"] / xcds)
            lines.append(f"  valu_busy: {busy:.3f}")
        if "SQ_VALU_MFMA_BUSY_CYCLES" in avg and "GRBM_GUI_ACTIVE" in avg:
            mb = avg["SQ_VALU_MFMA_BUSY_CYCLES"] / (simds * avg["GRBM_GUI_ACTIVE"] / xcds)
            lines.append(f"  mfma_busy: {mb:.4f}")
        if "SQ_INSTS_VALU_MFMA_MOPS_BF16" in avg:
            lines.append(f"  mfma_bf16_flop: {avg['SQ_INSTS_VALU_MFMA_MOPS_BF16'] * 512:.4g}")
        for prec in ("F32", "F64"):
            keys = [f"SQ_INSTS_VALU_{op}_{prec}" for op in ("ADD", "MUL", "FMA", "TRANS")]
            if all(k in avg for k in keys):
                # instructions count per wavefront: 64 lanes each; an FMA is 2 flops
                fl = 64.0 * (avg[keys[0]] + avg[keys[1]] + 2.0 * avg[keys[2]] + avg[keys[3]])
                lines.append(f"  valu_{prec.lower()}_flop: {fl:.6g}")
        if "SQ_WAIT_INST_ANY" in avg and "SQ_WAVE_CYCLES" in avg:
            lines.append(f"  wait_fraction: {avg['SQ_WAIT_INST_ANY'] / avg['SQ_WAVE_CYCLES']:.3f}")
        lines.append("")
    with open(out, "w") as f:
        f.write("\n".join(lines))


def read_traffic(path):
    """the key: value lines of a traffic summary, or None"""
    if not os.path.exists(path):
        return None
    d = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", " ")):
            k, v = line.split(":", 1)
            d[k.strip()] = v.strip()
    return d


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(*sys.argv[2:6])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]), sys.argv[6], sys.argv[7])
    elif sys.argv[1] == "counters":
        counters(sys.argv[2], sys.argv[3].split(";"), sys.argv[4], sys.argv[5])
    else:
        raise SystemExit(__doc__)
