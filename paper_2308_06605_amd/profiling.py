"""Turn rocprofv3 counter CSVs into per-kernel summaries.

HBM traffic (after two `rocprofv3 --pmc` runs of bench.py with --copy-calibration, one collecting
FETCH_SIZE and one WRITE_SIZE):

  python -m paper_2308_06605_amd.profiling --fetch <dir>/run_counter_collection.csv \\
      --write <dir>/run_counter_collection.csv --calib-bytes 268435456 --out <summary.json>

Other counters (any number of `--pmc` passes over the same command):

  python -m paper_2308_06605_amd.profiling counters <csv> [<csv> ...] --out <summary.md>

gives per kernel the mean of every counter over the kernel's dispatches and the derived ratios
the design notes use (VALU and LDS instructions per wave, LDS bank conflicts per LDS
instruction, waves resident per CU, LDS and VALU busy fractions).

Each counter is averaged per kernel over its dispatches (KiB per dispatch) and scaled by the
factor that makes the calibration copy (a plain device-to-device copy of --calib-bytes bytes)
read and write exactly that many bytes. The summary records a hash of the kernel sources, so a
reader can tell whether the counters still describe the current kernels.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# the sources each precision's stage kernels and their launchers are built from; of
# fr_kernels.hip only the part before its C ABI section (extern "C"), which holds the kernels
# and launchers, while the entry points after it do not change what a kernel does
KERNEL_SOURCES = {"fp64": ("fr_kernels.hip", "fr_device.h", "fr_internal.h"),
                  "fp32": ("fr_kernels32.hip", "fr_device.h", "fr_internal.h")}


def kernel_source_hash(prec: str = "fp64") -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[prec]:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            text = f.read()
        if name == "fr_kernels.hip":
            text = text.split(b'\nextern "C" {\n', 1)[0]
        h.update(text)
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """'void (anonymous namespace)::k_face32<3, true>(...)' -> 'k_face32'; a volume kernel's
    instance with the fused next-stage pre-pass (last template argument true) gets '_pre'
    ('k_volume_pre', 'k_volume32_pre')."""
    base = name.replace("void ", "").replace("(anonymous namespace)::", "")
    short = base.split("<")[0].split("(")[0].strip()
    if short in ("k_volume", "k_volume32") and "<" in base:
        targs = base.split("<", 1)[1].split(">")[0]
        if targs.split(",")[-1].strip() in ("true", "1"):
            return short + "_pre"
    return short


def per_kernel_kib(path: str, counter: str):
    vals = collections.defaultdict(list)
    grid = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            k = short_name(r["Kernel_Name"])
            vals[(k, r["Grid_Size"])].append(float(r["Counter_Value"]))
            grid[(k, r["Grid_Size"])] = int(r["Grid_Size"])
    return {key: sum(v) / len(v) for key, v in vals.items()}


def summarize(fetch_csv: str, write_csv: str, calib_bytes: int, prec: str = "fp64") -> dict:
    fetch = per_kernel_kib(fetch_csv, "FETCH_SIZE")
    write = per_kernel_kib(write_csv, "WRITE_SIZE")
    # the calibration copy: the copy dispatch with the largest write
    copies = [k for k in write if "copyBuffer" in k[0]]
    if not copies:
        raise SystemExit("no calibration copy dispatch found")
    cal = max(copies, key=lambda k: write[k])
    f_scale = calib_bytes / 1024.0 / fetch[cal]
    w_scale = calib_bytes / 1024.0 / write[cal]
    kernels = {}
    for key in fetch:
        name = key[0]
        if not name.startswith("k_") or key not in write:
            continue
        kernels[name] = {
            "fetch_bytes": fetch[key] * 1024.0 * f_scale,
            "write_bytes": write[key] * 1024.0 * w_scale,
        }
    return {"kernel_source_hash": kernel_source_hash(prec), "prec": prec, "fetch_scale": f_scale, "write_scale": w_scale,
            "calibration_copy_bytes": calib_bytes, "kernels": kernels}


def per_kernel_counters(paths):
    """{kernel: {counter: mean value per dispatch}} over the given counter-collection CSVs."""
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                k = short_name(r["Kernel_Name"])
                if not k.startswith("k_"):
                    continue
                vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in vals.items()}


def derived(c: dict) -> dict:
    """Ratios of one kernel's counters (per dispatch means); only those whose inputs exist."""
    out = {}
    w = c.get("SQ_WAVES")
    if w:
        for name in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
                     "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_MFMA"):
            if name in c:
                out[name.replace("SQ_INSTS_", "") + " per wave"] = c[name] / w
    if c.get("SQ_INSTS_LDS") and "SQ_LDS_BANK_CONFLICT" in c:
        out["LDS bank-conflict cycles per LDS instruction"] = c["SQ_LDS_BANK_CONFLICT"] / c["SQ_INSTS_LDS"]
    if c.get("SQ_BUSY_CYCLES") and "SQ_WAVE_CYCLES" in c:
        # wave-cycles summed over waves (counted per SE, in units of 4 cycles on this part) over
        # busy cycles: mean resident waves
        out["mean resident waves (wave cycles / busy cycles)"] = c["SQ_WAVE_CYCLES"] / c["SQ_BUSY_CYCLES"]
    for name in ("SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VALU", "SQ_WAIT_INST_LDS", "SQ_WAIT_ANY"):
        if name in c and c.get("SQ_WAVE_CYCLES"):
            out[name.replace("SQ_", "") + " / wave cycles"] = c[name] / c["SQ_WAVE_CYCLES"]
    return out


def counters_markdown(paths, title: str, command: str) -> str:
    data = per_kernel_counters(paths)
    lines = [f"# {title}", "", f"Command: `{command}`", "",
             "Mean per dispatch of each counter, then derived ratios.", ""]
    for k in sorted(data):
        lines.append(f"## {k}")
        lines.append("")
        lines.append("| counter | value |")
        lines.append("|---|---|")
        for name in sorted(data[k]):
            lines.append(f"| {name} | {data[k][name]:.6g} |")
        for name, v in derived(data[k]).items():
            lines.append(f"| *{name}* | {v:.4g} |")
        lines.append("")
    return "\n".join(lines)


def main():
    import sys

    if len(sys.argv) > 1 and sys.argv[1] == "counters":
        ap = argparse.ArgumentParser(prog="profiling counters")
        ap.add_argument("csv", nargs="+")
        ap.add_argument("--title", default="Kernel counters")
        ap.add_argument("--command", default="")
        ap.add_argument("--out", required=True)
        a = ap.parse_args(sys.argv[2:])
        text = counters_markdown(a.csv, a.title, a.command)
        with open(a.out, "w") as f:
            f.write(text + "\n")
        print(text)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--calib-bytes", type=int, required=True)
    ap.add_argument("--command", default="", help="the rocprofv3 command, recorded in the summary")
    ap.add_argument("--prec", choices=("fp64", "fp32"), default="fp64")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    s = summarize(a.fetch, a.write, a.calib_bytes, a.prec)
    s["command"] = a.command
    with open(a.out, "w") as f:
        json.dump(s, f, indent=1)
    print(json.dumps(s, indent=1))


if __name__ == "__main__":
    main()
