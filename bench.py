"""Benchmark: DOF-updates/s per RK stage of the FR residual + low-storage RK stage on one MI355X.

Default workload (the scaled-up plain-FR configuration): periodic 64^3 hexahedral box on
[0, 2 pi)^3 whose nodes are curved by 0.05 L sin(2 pi x/L) sin(2 pi y/L) sin(2 pi z/L)
(isoparametric, q = p = 3), Taylor-Green vortex at Mach 0.1 and Re 1600, Roe + BR2, the
Carpenter-Kennedy five-stage RK45 with dt = 2.5e-4, FP64. One bench step is one full RK step
(five stages); value = n_elem (p+1)^3 * stages / time.

Prints one JSON line (rank 0): metric, value, unit, timing and configuration fields, plus
`roofline` (HBM bound: the two-pass minimum bytes of one RK stage over the stage time measured
with HIP events on the launch stream, with the dominant kernel's own bytes over its mean launch
time as `dominant_kernel`), `variants` (the FP32 form at the same size, and 32^3 p=7 in both
precisions, timed the same way) and `cpu_baseline` (the CPU oracle timed on bounded samples).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2308_06605_amd.profiling import algorithmic_bytes, tile_elements  # noqa: E402 (the byte accounting)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
STAGES = {"lsrk45": 5, "rk4": 4}
KERNEL_NAMES = {"prepass": "k_prepass", "face": "k_face", "volume": "k_volume", "volume_pre": "k_volume_pre"}


def kernel_name(key: str, prec: str) -> str:
    """'volume_pre', 'fp32' -> 'k_volume32_pre' (the names the profiles use)"""
    if prec != "fp32":
        return KERNEL_NAMES[key]
    return "k_volume32_pre" if key == "volume_pre" else KERNEL_NAMES[key] + "32"


def make_workload(n: int, p: int, curved: bool):
    from paper_2308_06605_amd import inputs

    mesh = inputs.box_mesh(n, q=p, curve_amp=0.05 if curved else 0.0)
    return mesh


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_residual_rate(mesh, p, U, mu, flux, threads, n_sample):
    """DOF-updates/s of the oracle's residual on the first n_sample elements, a slab of whole
    element layers of the box (the oracle's subset mode also evaluates the traces of the
    sample's face neighbours: two more layers), median of 3 evaluations after 1 warm-up."""
    import oracle

    n = min(mesh.n_elem, int(n_sample))
    sample = np.arange(n, dtype=np.int64)
    o = oracle.Oracle(mesh, p, mu=mu, flux=flux, active=sample, nthreads=threads)
    o.residual(U)  # warm-up
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        o.residual(U)
        ts.append(time.perf_counter() - t0)
    return n * (p + 1) ** 3 / float(np.median(ts)), n


def cpu_baseline(mesh, p, U, mu, flux, extra=()):
    """The CPU oracle timed on this host: its residual (one RK stage's work) on a quarter of the
    benchmark mesh's elements, with the benchmark's state, on all threads (the reported value)
    and on two element layers with one thread; a full RK4 step on 8^3 p=3; and the residual of
    each extra (label, mesh, p, U) on a quarter of its elements."""
    import oracle

    from paper_2308_06605_amd import inputs

    threads = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        threads = min(threads, int(omp))
    E = mesh.n_elem
    layer = round(E ** (2 / 3))  # elements per layer of the n^3 box
    rate, n_sample = _oracle_residual_rate(mesh, p, U, mu, flux, threads, E // 4)
    rate1, n1 = _oracle_residual_rate(mesh, p, U, mu, flux, 1, 2 * layer)
    out = {"value": rate, "unit": "DOF-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"residual of the first {n_sample} elements (a quarter of the mesh, whole layers) "
                     f"of the same mesh and state, median of 3 after 1 warm-up, double precision, "
                     f"{threads} OpenMP threads",
           "cpu_model": _cpu_model(),
           "single_thread": {"value": rate1, "sample": f"residual of the first {n1} elements (two layers), "
                                                       f"1 thread"}}
    # ora_rk_step: one RK4 step (four residuals) of the whole 8^3 p=3 TGV
    m8 = inputs.box_mesh(8, q=1)
    o8 = oracle.Oracle(m8, 3, mu=mu, flux="rusanov", nthreads=threads)
    U8 = inputs.state_from_coords(o8.sol_coords(), inputs.tgv_state)
    o8.rk_step(U8, 1e-3, "rk4", 1)
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        o8.rk_step(U8, 1e-3, "rk4", 1)
        ts.append(time.perf_counter() - t0)
    out["rk_step_8cubed_p3"] = {"value": 4 * m8.n_elem * 64 / float(np.median(ts)), "unit": "DOF-updates/s",
                                "sample": "whole 8^3 p=3 TGV, one RK4 step (4 stages), median of 3"}
    for label, m, pp, UU in extra:
        r, ns = _oracle_residual_rate(m, pp, UU, mu, flux, threads, m.n_elem // 4)
        out[label] = {"value": r, "unit": "DOF-updates/s",
                      "sample": f"residual of the first {ns} elements (a quarter of the mesh)"}
    return out


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 3) -> float:
    """GB/s of a plain device-to-device copy of nbytes (read + write counted), median of reps,
    HIP events on the current stream: the practical HBM ceiling the roofline is also given
    against."""
    import torch

    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    del src, dst
    return 2 * nbytes / (float(np.median(ts)) * 1e-3) / 1e9


def run_config(fr, inputs, n, p, prec, args, mu, curved=True):
    """Build the curved TGV workload on n^3 elements at degree p in the given precision, pick
    tiles (autotuner or --tiles), run the warm-up and time args.steps RK steps with HIP events on
    the launch stream. Returns the timing record and (mesh, state) for the CPU baseline."""
    import torch

    mesh = make_workload(n, p, curved)
    t0 = time.perf_counter()
    p0 = 1.0 / (1.4 * 0.1 * 0.1)  # TGV reference pressure at Mach 0.1
    g = fr.FRMesh(mesh, p, mu=mu, flux=args.flux, prec=prec, ref_rho=1.0, ref_p=p0)
    t_setup = time.perf_counter() - t0
    U = inputs.state_from_coords(g.sol_coords(), inputs.tgv_state)
    g.set_state(U)
    torch.cuda.synchronize()
    tile_ms = None
    if args.tiles is not None:
        g.set_tiles(*args.tiles)
        if args.fuse is not None:
            g.set_fusion(bool(args.fuse))
    else:
        _, tile_ms = g.autotune(2)
    tiles, fused = g.tiles(), g.fusion()
    stages = STAGES[args.scheme]
    for _ in range(args.warmup):
        g.rk_step(args.dt, args.scheme, 1)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    g.rk_step(args.dt, args.scheme, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_step = e0.elapsed_time(e1) / args.steps
    # the same K steps repeated (not part of `value`), and the residual alone
    repeats = []
    for _ in range(args.repeats):
        e0.record(stream)
        g.rk_step(args.dt, args.scheme, args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        repeats.append(e0.elapsed_time(e1) / args.steps)
    Rt = torch.empty((mesh.n_elem, 5, (p + 1) ** 3), dtype=torch.float64, device="cuda")
    res_ms = []
    for _ in range(1 + args.repeats):
        e0.record(stream)
        g.residual(out=Rt)
        e1.record(stream)
        torch.cuda.synchronize()
        res_ms.append(e0.elapsed_time(e1))
    del Rt
    dof = mesh.n_elem * (p + 1) ** 3
    stage_ms = ms_step / stages
    # per-kernel mean launch durations (HIP events on the launch stream); with fusion the
    # pre-pass runs once per run of stages and every other stage is face + volume_pre
    kms = {k: v for k, v in g.profile_stages(args.dt, args.scheme, 2).items() if v > 0}
    ab = algorithmic_bytes(p, prec, affine=not curved)
    E = mesh.n_elem
    gbs = {k: ab[k] * E / (kms[k] * 1e-3) / 1e9 for k in kms}
    per_stage = ("face", "volume_pre") if "volume_pre" in kms else ("prepass", "face", "volume")
    dominant = max(per_stage, key=kms.get)
    stage_bytes = ab["stage_min"] * E
    stage_gbs = stage_bytes / (stage_ms * 1e-3) / 1e9
    finite = bool(np.isfinite(g.get_state()).all())
    g.close()

    # measured HBM traffic of the stage's kernels from the committed rocprofv3 summary, only
    # while the kernel sources still match the ones the counters were taken on
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_n{n}_p{p}_{prec}{'' if curved else '_affine'}.json")
    if os.path.exists(tfile):
        from paper_2308_06605_amd import profiling

        with open(tfile) as f:
            ts = json.load(f)
        recs = [ts["kernels"].get(kernel_name(k, prec)) for k in per_stage]
        if ts.get("kernel_source_hash") == profiling.kernel_source_hash(prec) and all(recs):
            traffic = sum(r["fetch_bytes"] + r["write_bytes"] for r in recs)
    return {
        "workload": (f"TGV Ma0.1 Re1600, {'curved' if curved else 'affine'} periodic {n}^3 hex, p={p}, "
                     f"{args.flux.capitalize()}+BR2, {args.scheme.upper()} dt={args.dt}, "
                     f"{'FP64' if prec == 'fp64' else 'FP32 operators/fluxes, FP64 state and mass'}"),
        "n": n, "n_elem": E, "dof": dof, "p": p, "prec": prec,
        "value": dof * stages / (ms_step * 1e-3), "ms_per_step": ms_step, "stage_ms": stage_ms,
        "repeats_ms_per_step": repeats,
        "median_value": dof * stages / (float(np.median([ms_step, *repeats])) * 1e-3),
        "residual_ms": float(np.median(res_ms[1:])) if len(res_ms) > 1 else res_ms[0],
        "tiles": {"elements_per_block": tile_elements(p, tiles[0]), "epb_choice": int(tiles[0]),
                  "face_block": (256, 128, 64)[tiles[1]], "fused_prepass": fused,
                  "autotune_ms_per_stage": None if tile_ms is None else [float(x) for x in tile_ms]},
        "roofline": {"bound": "hbm", "achieved": stage_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": stage_gbs / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": " + ".join(kernel_name(k, prec) for k in per_stage) + " (one RK stage)",
                     "bytes_per_stage": stage_bytes,
                     "bytes_rule": {("fp64", True): "8 (45 Ns + 44 Nf) per element",
                                    ("fp32", True): "8 * 25 Ns + 4 (20 Ns + 44 Nf) per element",
                                    ("fp64", False): "8 (25 Ns + 40 Nf) per element (affine elements)",
                                    ("fp32", False): "8 * 25 Ns + 4 * 40 Nf per element (affine elements)"}[(prec, curved)],
                     "dominant_kernel": {"kernel": kernel_name(dominant, prec),
                                         "bytes_per_launch": ab[dominant] * E,
                                         "mean_launch_ms": kms[dominant],
                                         "achieved": gbs[dominant],
                                         "frac": gbs[dominant] / HBM_PEAK_GBS}},
        "kernel_ms": kms, "kernel_gbs": gbs, "setup_s": t_setup, "wall_s_timed": t_wall, "finite": finite,
        "_mesh": mesh, "_U": U,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=64, help="elements per direction")
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--affine", action="store_true", help="uncurved mesh")
    ap.add_argument("--flux", default="roe")
    ap.add_argument("--scheme", default="lsrk45")
    ap.add_argument("--dt", type=float, default=2.5e-4)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32"],
                    help="fp32: FP32 operators and fluxes with FP64 state and mass equation")
    ap.add_argument("--tiles", type=int, nargs=2, default=None, metavar=("EPB", "FBS"),
                    help="fixed tile shapes (fr_set_tiles) instead of running the autotuner")
    ap.add_argument("--fuse", type=int, choices=(0, 1), default=None,
                    help="with --tiles: the fused pre-pass on (1, the default) or off (fr_set_fusion)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the other precision and degree (FP32 form at this size, 32^3 p=7 in both)")
    ap.add_argument("--repeats", type=int, default=4,
                    help="repeat the K timed steps this many more times (median_value; not `value`)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-sized device buffer once (a known-size "
                         "dispatch that scales the profiler's FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (one process, one device); "
                                   "--gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2308_06605_amd import fr, inputs

    torch.cuda.set_device(0)
    mu = 1.0 / 1600.0
    curved = not args.affine
    main_run = run_config(fr, inputs, args.n, args.p, args.prec, args, mu, curved)
    mesh, U = main_run.pop("_mesh"), main_run.pop("_U")
    cgbs = copy_bandwidth()
    main_run["roofline"]["copy_gbs"] = cgbs
    main_run["roofline"]["frac_of_copy"] = main_run["roofline"]["achieved"] / cgbs

    variants = {}
    p7 = None
    if not args.no_variants:
        other = "fp32" if args.prec == "fp64" else "fp64"
        plan = [(other, args.n, args.p)]
        plan = [(prec, n, p, curved) for prec, n, p in plan]
        if args.p == 3 and args.n == 64:
            # the precision variant's p = 7 workload, 32^3 (the same 16.8M DOF), in both forms,
            # and the uniform (affine) 64^3 box in FP64
            plan += [("fp64", 32, 7, curved), ("fp32", 32, 7, curved)]
            if curved:
                plan += [("fp64", 64, 3, False)]
        for prec, n, p, cv in plan:
            r = run_config(fr, inputs, n, p, prec, args, mu, cv)
            m7, U7 = r.pop("_mesh"), r.pop("_U")
            if p == 7 and p7 is None:
                p7 = (m7, U7)
            r["speedup_vs_fp64_same_size"] = None
            variants[f"{prec}_n{n}_p{p}" + ("" if cv == curved else "_affine")] = r
        runs = [main_run, *variants.values()]
        for r in variants.values():
            ref = [q for q in runs if (q["n"], q["p"], q["prec"], q["workload"].split(",")[1])
                   == (r["n"], r["p"], "fp64", r["workload"].split(",")[1])]
            if r["prec"] == "fp32" and ref:
                ref = ref[0]
                r["speedup_vs_fp64_same_size"] = ref["ms_per_step"] / r["ms_per_step"]

    cpu = None
    if not args.no_cpu:
        try:
            extra = [("residual_32cubed_p7", p7[0], 7, p7[1])] if p7 is not None else []
            cpu = cpu_baseline(mesh, args.p, U, mu, args.flux, extra)
        except Exception as exc:  # report, never fake
            cpu = {"error": str(exc)}

    out = {
        "metric": "DOF-updates/s per RK stage",
        "value": main_run["value"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": main_run["workload"], "n_elem": main_run["n_elem"], "dof": main_run["dof"],
                   "p": args.p, "tiles": main_run["tiles"], "stages_per_step": STAGES[args.scheme],
                   "parallelism": "single GPU"},
        "roofline": main_run["roofline"],
        "stage": {k: main_run[k] for k in ("stage_ms", "kernel_ms", "kernel_gbs", "repeats_ms_per_step",
                                           "median_value", "residual_ms")},
        "variants": variants,
        "cpu_baseline": cpu,
        "setup_s": main_run["setup_s"],
        "wall_s_timed": main_run["wall_s_timed"],
        "finite": main_run["finite"] and all(v["finite"] for v in variants.values()),
    }
    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = n * 8
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
