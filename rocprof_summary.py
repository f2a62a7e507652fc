"""Summaries of rocprofv3 CSV output for the H*psi kernels.

    python rocprof_summary.py trace  DIR             # --kernel-trace --stats run
    python rocprof_summary.py traffic FETCH_DIR WRITE_DIR HPSI_LAUNCHES COPY_MIB OUT.json
    python rocprof_summary.py counters DIR HPSI_LAUNCHES OUT.json [ALGORITHMIC_FLOPS]

`counters` sums every counter of one --pmc run over the last HPSI_LAUNCHES
dispatches of the BF16 grouped GEMMs (executed MFMA flops = 512 per
SQ_INSTS_VALU_MFMA_MOPS_BF16 MOP) and writes them to OUT.json with the
kernel source hash.

`trace` prints per-kernel totals of the run and the kernels of its last BF16
H*psi (bench.py times one BF16 and one FP64 H*psi per step).

`traffic` reads two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of
`bench.py --copy-calibration MIB`.  Each counter is scaled by what it reads
for the plain device copy of known size (bytes copied / counter bytes), and
the HBM bytes of the dominant kernels -- the BF16 grouped GEMMs
gemm_bf16_pipe, gemm_bf16_padded and gemm_bf16_wave -- over the last BF16 H*psi of the run
(its last HPSI_LAUNCHES dispatches of them) are written to OUT.json together
with the SHA-256 of the kernel source, so that a later reader can tell whether
the figures still describe the kernel.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

KERNEL_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2503_20700_amd", "csrc", "exec_hip.hip")


def source_sha256() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


BF16_GEMMS = ("gemm_bf16_padded", "gemm_bf16_wave", "gemm_bf16_pipe")


def short_name(name: str) -> str:
    m = re.search(r"(gemm_kernel|gemm_bf16_padded|gemm_bf16_pipe|gemm_bf16_wave|gemm_f64_pipe|gemm_f64_wave|reduce_kernel|"
                  r"convert_kernel|"
                  r"pack_kernel)"
                  r"<([^>]*)>", name)
    if m:
        return f"{m.group(1)}<{m.group(2)}>"
    return name.split("(")[0][:60]


def _rows(path):
    with open(path) as f:
        return list(csv.DictReader(f))


def trace(d: str) -> None:
    rows = _rows(os.path.join(d, "run_kernel_trace.csv"))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    tot = defaultdict(lambda: [0, 0.0])
    for r in rows:
        a = tot[short_name(r["Kernel_Name"])]
        a[0] += 1
        a[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
    print("| kernel | calls | total ms | avg us |\n|---|---|---|---|")
    for k, (n, ms) in sorted(tot.items(), key=lambda x: -x[1][1])[:12]:
        print(f"| {k} | {n} | {ms:.1f} | {ms / n * 1e3:.1f} |")
    # last BF16 H*psi: the final run of consecutive BF16 grouped GEMM / reduce launches
    names = [short_name(r["Kernel_Name"]) for r in rows]
    last = max(i for i, n in enumerate(names) if n.startswith(BF16_GEMMS))
    first = last
    while first > 0 and (names[first - 1].startswith(BF16_GEMMS) or names[first - 1].startswith("reduce_kernel<1")):
        first -= 1
    grp = defaultdict(lambda: [0, 0.0, 0])
    for r in rows[first:last + 1]:
        a = grp[short_name(r["Kernel_Name"])]
        a[0] += 1
        a[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        a[2] += int(r["Grid_Size_X"]) // 256
    print("\nLast BF16 H*psi:\n\n| kernel | launches | total ms | avg us | work-groups / launch |\n|---|---|---|---|---|")
    for k, (n, ms, wg) in grp.items():
        print(f"| {k} | {n} | {ms:.1f} | {ms / n * 1e3:.1f} | {wg / n:.0f} |")
    span = (int(rows[last]["End_Timestamp"]) - int(rows[first]["Start_Timestamp"])) / 1e6
    print(f"\nwindow {span:.1f} ms")


def _counter(rows, kernel_pred):
    out = []
    for r in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
        if kernel_pred(r["Kernel_Name"]):
            out.append(float(r["Counter_Value"]) * 1024.0)  # KiB -> bytes
    return out


def traffic(fetch_dir: str, write_dir: str, launches: int) -> dict:
    res = {"kernel": "+".join(BF16_GEMMS), "source_sha256": source_sha256(), "launches": launches}
    for name, d in (("fetch", fetch_dir), ("write", write_dir)):
        rows = _rows(os.path.join(d, "run_counter_collection.csv"))
        # the calibration copy is the largest copyBuffer dispatch of the run
        counted = max(_counter(rows, lambda n: "copyBuffer" in n))
        gem = _counter(rows, lambda n: any(k in n for k in BF16_GEMMS))
        res[name] = {"copy_counter_bytes": counted, "gemm_counter_bytes_last_hpsi": sum(gem[-launches:])}
    return res


def counters(d: str, launches: int) -> dict:
    """Per-counter sums over the last `launches` dispatches of the BF16 grouped
    GEMMs in one --pmc run (several counters per dispatch)."""
    rows = _rows(os.path.join(d, "run_counter_collection.csv"))
    by_dispatch = defaultdict(dict)
    name_of = {}
    for r in rows:
        di = int(r["Dispatch_Id"])
        by_dispatch[di][r["Counter_Name"]] = by_dispatch[di].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        name_of[di] = r["Kernel_Name"]
    gem = [di for di in sorted(by_dispatch) if any(k in name_of[di] for k in BF16_GEMMS)]
    sel = gem[-launches:]
    out = defaultdict(float)
    for di in sel:
        for k, v in by_dispatch[di].items():
            out[k] += v
    return {"kernel": "+".join(BF16_GEMMS), "source_sha256": source_sha256(), "launches": len(sel),
            "counters": dict(out)}


def main(argv):
    if len(argv) >= 4 and argv[0] == "counters":
        # counters DIR HPSI_LAUNCHES OUT.json [ALGORITHMIC_FLOPS]
        res = counters(argv[1], int(argv[2]))
        c = res["counters"]
        if "SQ_INSTS_VALU_MFMA_MOPS_BF16" in c:
            # one MOP is 512 floating-point operations of a BF16 MFMA
            res["mfma_flops_executed"] = c["SQ_INSTS_VALU_MFMA_MOPS_BF16"] * 512.0
            if len(argv) >= 5:
                res["algorithmic_flops"] = float(argv[4])
                res["executed_over_algorithmic"] = res["mfma_flops_executed"] / res["algorithmic_flops"]
        if "SQ_VALU_MFMA_BUSY_CYCLES" in c and c.get("GRBM_GUI_ACTIVE"):
            # GRBM_GUI_ACTIVE is summed over the 8 XCDs; 256 CUs x 4 SIMDs
            res["mfma_busy_fraction"] = c["SQ_VALU_MFMA_BUSY_CYCLES"] / (c["GRBM_GUI_ACTIVE"] / 8.0 * 1024.0)
            res["note"] = ("GRBM_GUI_ACTIVE is summed over the 8 XCDs (per-XCD active cycles = sum / 8); MFMA busy = "
                           "SQ_VALU_MFMA_BUSY_CYCLES / (per-XCD active cycles x 1024 SIMDs)")
        with open(argv[3], "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res, indent=1))
        return 0
    if len(argv) >= 2 and argv[0] == "trace":
        trace(argv[1])
        return 0
    if len(argv) >= 6 and argv[0] == "traffic":
        fetch_dir, write_dir, launches, copy_mib, out_path = argv[1], argv[2], int(argv[3]), int(argv[4]), argv[5]
        res = traffic(fetch_dir, write_dir, launches)
        copied = copy_mib * 1024.0 * 1024.0
        total = 0.0
        for name in ("fetch", "write"):
            r = res[name]
            r["scale"] = copied / r["copy_counter_bytes"]
            r["hbm_bytes_last_hpsi"] = r["gemm_counter_bytes_last_hpsi"] * r["scale"]
            total += r["hbm_bytes_last_hpsi"]
        res["copy_mib"] = copy_mib
        res["hbm_bytes_per_hpsi"] = total
        with open(out_path, "w") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res, indent=1))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
