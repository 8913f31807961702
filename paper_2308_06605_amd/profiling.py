"""Turn rocprofv3 counter CSVs into per-kernel summaries.

HBM traffic (after two `rocprofv3 --pmc` runs of bench.py with --copy-calibration, one collecting
FETCH_SIZE and one WRITE_SIZE):

  python -m paper_2308_06605_amd.profiling --fetch <dir>/run_counter_collection.csv \\
      --write <dir>/run_counter_collection.csv --calib-bytes 268435456 --out <summary.json>

The stage summary of a workload (a `rocprofv3 --kernel-trace --stats` run and the traffic JSON):

  python -m paper_2308_06605_amd.profiling stage --stats <dir>/run_kernel_stats.csv \\
      --traffic <traffic.json> --n 64 --p 3 --prec fp64 --tiles 0 2 --fuse 1 --command "<cmd>" --out <md>

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


def algorithmic_bytes(p: int, prec: str = "fp64", viscous: bool = True, affine: bool = False):
    """HBM bytes per element per stage that each kernel must move (every input read once,
    every output written once); the state and RK registers are always FP64.

    pre-pass : read U (5 Ns) and volume geometry (10 Ns); write own face data (20 Nf)
    face     : per face point read both sides' face data (2 x 20) and the face geometry (4),
               write the jump and common flux (10); per element that is 3 Nfp points
    volume   : read U (5 Ns), the volume geometry (10 Ns), its faces' jumps and fluxes (10 Nf)
               and the RK register (5 Ns); write the register (5 Ns) and U (5 Ns): 30 Ns + 10 Nf
               (an LSRK45 run's first stage reads no register: 25 Ns)
    volume_pre : the volume kernel that also runs the next stage's pre-pass on the state it
               stores: the volume kernel's bytes plus the pre-pass's writes (FP64 20 Nf doubles;
               FP32 form 20 Nf floats + 3 Nf doubles); its reads of U and the geometry are the
               volume kernel's own
    In the FP64 path a stage is face + volume_pre, 8 (30 Ns + 57 Nf) per element: 924 B/DOF at
    p = 3. `stage_min` is the two-pass minimum of a stage that reads its inputs in both passes:
    FP64 8 (45 Ns + 44 Nf); FP32 form (FP64 state, FP32 geometry and face data)
    8 * 25 Ns + 4 (20 Ns + 44 Nf). The roofline of the whole stage is taken on it.
    affine: the two-pass minimum of a mesh of affine elements, whose metric terms and face
    normals are constant per element and face: FP64 8 (25 Ns + 40 Nf) (680 B/DOF at p = 3), FP32
    form 8 * 25 Ns + 4 * 40 Nf. The kernels' own bytes do not change: they read the terms per
    point on every mesh.
    """
    n = p + 1
    Ns, Nfp = n ** 3, n * n
    Nf = 6 * Nfp
    nv = 20 if viscous else 5
    if prec == "fp64":
        k1 = 8 * 5 * Ns + 8 * (10 * Ns + nv * Nf)
        k2 = 8 * 3 * Nfp * (2 * nv + 4 + 10)
        k3 = 8 * 20 * Ns + 8 * (10 * Ns + 10 * Nf)
        stage_min = 8 * (45 * Ns + 44 * Nf)
    else:
        # FP32 form: FP32 geometry copy for the pre-pass, face data as 20 floats + 3 doubles,
        # face results as 9 floats + 1 double; the volume kernel reads FP64 geometry (mass)
        k1 = 8 * 5 * Ns + 4 * 10 * Ns + (4 * nv + 8 * 3) * Nf
        k2 = 3 * Nfp * (2 * (4 * nv + 8 * 3) + 8 * 4 + 4 * 9 + 8)
        k3 = 8 * 20 * Ns + 8 * 10 * Ns + (4 * 9 + 8) * Nf
        stage_min = 8 * 25 * Ns + 4 * (20 * Ns + 44 * Nf)
    if affine:
        stage_min = 8 * (25 * Ns + 40 * Nf) if prec == "fp64" else 8 * 25 * Ns + 4 * 40 * Nf
    out = {"prepass": k1, "face": k2, "volume": k3, "stage_min": stage_min}
    # the volume kernel with the next stage's pre-pass adds the pre-pass's writes
    out["volume_pre"] = k3 + (8 * nv * Nf if prec == "fp64" else (4 * nv + 8 * 3) * Nf)
    return out


def tile_elements(p: int, epb: int) -> int:
    """Elements per block of the element kernels for tile choice epb (0 or 1) at degree p: 256/Ns
    (at least one, at most 64), then half of it, or two where one element leaves lanes of its
    last wave idle (p = 5, 6)."""
    ns = (p + 1) ** 3
    e0 = min(64, max(1, 256 // ns))
    if epb == 0:
        return e0
    return e0 // 2 if e0 > 1 else (2 if ns % 64 and 2 * ns <= 1024 else 1)


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


def last_copy_kib(path: str, counter: str) -> float:
    """The counter of the run's last device copy: the calibration copy bench.py makes after
    everything else (other copies, such as state uploads and the copy-bandwidth measurement, share
    its kernel and grid size, so it is told apart by dispatch order)."""
    last = None
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]:
                d = int(r["Dispatch_Id"])
                if last is None or d > last[0]:
                    last = (d, float(r["Counter_Value"]))
    if last is None:
        raise SystemExit("no calibration copy dispatch found")
    return last[1]


def summarize(fetch_csv: str, write_csv: str, calib_bytes: int, prec: str = "fp64") -> dict:
    fetch = per_kernel_kib(fetch_csv, "FETCH_SIZE")
    write = per_kernel_kib(write_csv, "WRITE_SIZE")
    f_scale = calib_bytes / 1024.0 / last_copy_kib(fetch_csv, "FETCH_SIZE")
    w_scale = calib_bytes / 1024.0 / last_copy_kib(write_csv, "WRITE_SIZE")
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


def kernel_stats(path: str) -> dict:
    """{short kernel name: (calls, avg ms, min ms, max ms)} from rocprofv3's kernel_stats.csv."""
    out = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            k = short_name(r["Name"])
            if not k.startswith("k_"):
                continue
            out[k] = (int(r["Calls"]), float(r["AverageNs"]) * 1e-6, float(r["MinNs"]) * 1e-6,
                      float(r["MaxNs"]) * 1e-6)
    return out


def stage_markdown(stats_csv: str, traffic_json: str, n: int, p: int, prec: str, tiles, fuse: bool,
                   trace_command: str) -> str:
    """The stage summary of one workload: per kernel the profiler's launch times, the algorithmic
    bytes per launch (algorithmic_bytes times the element count) and the counters' HBM bytes."""
    st = kernel_stats(stats_csv)
    with open(traffic_json) as f:
        tr = json.load(f)
    E = n ** 3
    ab = algorithmic_bytes(p, prec)
    kinds = {"prepass": "k_prepass", "face": "k_face", "volume": "k_volume", "volume_pre": "k_volume_pre"}
    if prec == "fp32":
        kinds = {k: ("k_volume32_pre" if k == "volume_pre" else v + "32") for k, v in kinds.items()}
    epb = f"{tile_elements(p, tiles[0])} elements"
    fbs = (256, 128, 64)[tiles[1]]
    src = kernel_source_hash(prec)
    lines = [f"# Stage kernels, {n}^3 p={p} curved TGV (Roe+BR2, LSRK45), {prec.upper()}", "",
             f"Kernel trace: `{trace_command}` (tiles (elements per block, face block) = ({epb}, {fbs}), "
             f"fused pre-pass {'on' if fuse else 'off'}).", "",
             f"Traffic: `{tr.get('command', '')}`; FETCH_SIZE scaled by {tr['fetch_scale']:.4f}, WRITE_SIZE by "
             f"{tr['write_scale']:.4f} (the factors that make a {tr['calibration_copy_bytes'] >> 20} MiB device copy "
             f"read and write that many bytes). Counters taken on kernel sources {tr['kernel_source_hash']}; "
             f"the trace on {src}" + (" (same)." if src == tr["kernel_source_hash"] else " (the counters are stale)."),
             "", "| kernel | calls | avg ms | min ms | max ms | algorithmic GB/launch | measured HBM GB/launch "
             "(read + write) | algorithmic GB/s at avg | measured GB/s at avg |", "|---|---|---|---|---|---|---|---|---|"]
    for kind, name in kinds.items():
        if name not in st:
            continue
        calls, avg, mn, mx = st[name]
        alg = ab[kind] * E / 1e9
        k = tr["kernels"].get(name)
        rd, wr = (k["fetch_bytes"] / 1e9, k["write_bytes"] / 1e9) if k else (float("nan"), float("nan"))
        lines.append(f"| {name} | {calls} | {avg:.4f} | {mn:.4f} | {mx:.4f} | {alg:.3f} | {rd:.3f} + {wr:.3f} | "
                     f"{alg / avg * 1e3:.0f} | {(rd + wr) / avg * 1e3:.0f} |")
    # a stage: the face kernel and the fused volume kernel, or without fusion the three kernels
    parts = [kinds["face"], kinds["volume_pre"]] if fuse else [kinds["prepass"], kinds["face"], kinds["volume"]]
    if all(k in st for k in parts):
        t = sum(st[k][1] for k in parts)
        smin = ab["stage_min"] * E
        lines += ["", f"Stage ({' + '.join(parts)}): {t:.4f} ms, {n ** 3 * (p + 1) ** 3 / (t * 1e-3):.4g} DOF-updates/s; "
                  f"two-pass minimum {smin / 1e9:.3f} GB per stage, {smin / (t * 1e-3) / 1e9:.0f} GB/s, "
                  f"{smin / (t * 1e-3) / 8e12:.3f} of 8 TB/s."]
    return "\n".join(lines) + "\n"


def main():
    import sys

    if len(sys.argv) > 1 and sys.argv[1] == "stage":
        ap = argparse.ArgumentParser(prog="profiling stage")
        ap.add_argument("--stats", required=True, help="rocprofv3 --stats kernel_stats.csv")
        ap.add_argument("--traffic", required=True, help="the traffic summary JSON of the same workload")
        ap.add_argument("--n", type=int, required=True)
        ap.add_argument("--p", type=int, required=True)
        ap.add_argument("--prec", choices=("fp64", "fp32"), required=True)
        ap.add_argument("--tiles", type=int, nargs=2, required=True)
        ap.add_argument("--fuse", type=int, choices=(0, 1), required=True)
        ap.add_argument("--command", required=True, help="the kernel-trace command, recorded")
        ap.add_argument("--out", required=True)
        a = ap.parse_args(sys.argv[2:])
        text = stage_markdown(a.stats, a.traffic, a.n, a.p, a.prec, a.tiles, bool(a.fuse), a.command)
        with open(a.out, "w") as f:
            f.write(text)
        print(text)
        return
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
