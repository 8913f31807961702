"""Benchmark: DOF-updates/s per RK stage of the FR residual + low-storage RK stage on one MI355X.

Default workload (the scaled-up plain-FR configuration): periodic 64^3 hexahedral box on
[0, 2 pi)^3 whose nodes are curved by 0.05 L sin(2 pi x/L) sin(2 pi y/L) sin(2 pi z/L)
(isoparametric, q = p = 3), Taylor-Green vortex at Mach 0.1 and Re 1600, Roe + BR2, the
Carpenter-Kennedy five-stage RK45 with dt = 2.5e-4, FP64. One bench step is one full RK step
(five stages); value = n_elem (p+1)^3 * stages / time.

Prints one JSON line (rank 0): metric, value, unit, timing and configuration fields, plus
`roofline` (dominant kernel, HBM
bound, algorithmic bytes per launch over its mean launch time measured with HIP events on the
launch stream) and `cpu_baseline` (the CPU oracle timed on a bounded element sample).
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
STAGES = {"lsrk45": 5, "rk4": 4}
KERNEL_NAMES = {"prepass": "k_prepass", "face": "k_face", "volume": "k_volume", "volume_pre": "k_volume_pre"}


def kernel_name(key: str, prec: str) -> str:
    """'volume_pre', 'fp32' -> 'k_volume32_pre' (the names the profiles use)"""
    if prec != "fp32":
        return KERNEL_NAMES[key]
    return "k_volume32_pre" if key == "volume_pre" else KERNEL_NAMES[key] + "32"


def algorithmic_bytes(p: int, prec: str = "fp64", viscous: bool = True):
    """HBM bytes per element per stage that each kernel must move (every input read once,
    every output written once); the state and RK register are always FP64.

    pre-pass : read U (5 Ns) and volume geometry (10 Ns); write own face data (20 Nf)
    face     : per face point read both sides' face data (2 x 20) and the face geometry (4),
               write the jump and common flux (10); per element that is 3 Nfp points
    volume   : read U (5 Ns), volume geometry (10 Ns), its faces' jumps and fluxes (10 Nf) and
               dU (5 Ns); write dU (5 Ns) and U (5 Ns)
    volume_pre : the volume kernel that also runs the next stage's pre-pass on the state it
               stores: the volume kernel's bytes plus the pre-pass's writes (FP64 20 Nf doubles;
               FP32 form 20 Nf floats + 3 Nf doubles); its reads of U and the geometry are the
               volume kernel's own
    In the FP64 path a stage is face + volume_pre, 8 (25 Ns + 57 Nf) per element. The stage
    minimum of a two-pass design that reads its inputs in both passes is 8 (45 Ns + 44 Nf);
    `stage_min` returns that figure for the roofline of the whole stage.
    """
    n = p + 1
    Ns, Nfp = n ** 3, n * n
    Nf = 6 * Nfp
    nv = 20 if viscous else 5
    if prec == "fp64":
        k1 = 8 * 5 * Ns + 8 * (10 * Ns + nv * Nf)
        k2 = 8 * 3 * Nfp * (2 * nv + 4 + 10)
        k3 = 8 * 15 * Ns + 8 * (10 * Ns + 10 * Nf)
    else:
        # FP32 form: FP32 geometry copy for the pre-pass, face data as 20 floats + 3 doubles,
        # face results as 9 floats + 1 double; the volume kernel reads FP64 geometry (mass)
        k1 = 8 * 5 * Ns + 4 * 10 * Ns + (4 * nv + 8 * 3) * Nf
        k2 = 3 * Nfp * (2 * (4 * nv + 8 * 3) + 8 * 4 + 4 * 9 + 8)
        k3 = 8 * 15 * Ns + 8 * 10 * Ns + (4 * 9 + 8) * Nf
    stage_min = 8 * (45 * Ns + 44 * Nf)
    out = {"prepass": k1, "face": k2, "volume": k3, "stage_min": stage_min}
    # the volume kernel with the next stage's pre-pass adds the pre-pass's writes
    out["volume_pre"] = k3 + (8 * nv * Nf if prec == "fp64" else (4 * nv + 8 * 3) * Nf)
    return out


def make_workload(n: int, p: int, curved: bool):
    from paper_2308_06605_amd import inputs

    mesh = inputs.box_mesh(n, q=p, curve_amp=0.05 if curved else 0.0)
    return mesh


def cpu_baseline(mesh, p, U, mu, flux, target_s=12.0):
    """Time the CPU oracle's residual (one RK stage's work) on a bounded element sample."""
    import oracle

    threads = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp:
        threads = min(threads, int(omp))
    rng = np.random.default_rng(0)
    E = mesh.n_elem
    n_probe = min(E, 512)
    probe = np.sort(rng.choice(E, size=n_probe, replace=False))
    o = oracle.Oracle(mesh, p, mu=mu, flux=flux, active=probe, nthreads=threads)
    o.residual(U)  # warm-up
    t0 = time.perf_counter()
    o.residual(U)
    t_probe = time.perf_counter() - t0
    n_sample = int(min(E, max(n_probe, n_probe * target_s / 3 / max(t_probe, 1e-6))))
    sample = np.sort(rng.choice(E, size=n_sample, replace=False))
    o = oracle.Oracle(mesh, p, mu=mu, flux=flux, active=sample, nthreads=threads)
    o.residual(U)
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        o.residual(U)
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    dof = n_sample * (p + 1) ** 3
    return {"value": dof / t, "unit": "DOF-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"residual of {n_sample} random elements of the same mesh and state "
                      f"(median of 3 after 1 warm-up), double precision, {threads} OpenMP threads"}


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
    ap.add_argument("--no-variants", action="store_true", help="skip timing the FP32 form")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-sized device buffer once (a known-size "
                         "dispatch that scales the profiler's FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    from paper_2308_06605_amd import fr, inputs

    torch.cuda.set_device(0)
    mu = 1.0 / 1600.0
    mesh = make_workload(args.n, args.p, not args.affine)
    t0 = time.perf_counter()
    p0 = 1.0 / (1.4 * 0.1 * 0.1)  # TGV reference pressure at Mach 0.1
    g = fr.FRMesh(mesh, args.p, mu=mu, flux=args.flux, prec=args.prec, ref_rho=1.0, ref_p=p0)
    t_setup = time.perf_counter() - t0
    X = g.sol_coords()
    U = inputs.state_from_coords(X, inputs.tgv_state)
    g.set_state(U)
    torch.cuda.synchronize()
    # tile shapes and the fused pre-pass: the autotuner's choice on this mesh, or fixed ones
    tile_ms = None
    if args.tiles is not None:
        g.set_tiles(*args.tiles)
        if args.fuse is not None:
            g.set_fusion(bool(args.fuse))
    else:
        _, tile_ms = g.autotune(2)
    tiles = g.tiles()
    fused = g.fusion()

    stages = STAGES[args.scheme]
    for _ in range(args.warmup):
        g.rk_step(args.dt, args.scheme, 1)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    g.rk_step(args.dt, args.scheme, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    dof = mesh.n_elem * (args.p + 1) ** 3
    value = dof * stages / (ms_step * 1e-3)

    # per-kernel mean launch durations (HIP events on the launch stream)
    # (FP64: the pre-pass runs once per run of stages, every other stage is face + volume_pre)
    kms = {k: v for k, v in g.profile_stages(args.dt, args.scheme, 2).items() if v > 0}
    ab = algorithmic_bytes(args.p, args.prec)
    gbs = {k: ab[k] * mesh.n_elem / (kms[k] * 1e-3) / 1e9 for k in kms}
    per_stage = ("face", "volume_pre") if "volume_pre" in kms else ("prepass", "face", "volume")
    dominant = max(per_stage, key=kms.get)
    achieved = gbs[dominant]
    stage_ms = ms_step / stages
    stage_bytes = ab["stage_min"] * mesh.n_elem
    ok = bool(np.isfinite(g.get_state()).all())

    # HBM traffic of the dominant kernel from the committed rocprofv3 summary, only while the
    # kernel sources still match the ones the counters were taken on
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_n{args.n}_p{args.p}_{args.prec}"
                         f"{'_affine' if args.affine else ''}.json")
    if os.path.exists(tfile):
        from paper_2308_06605_amd import profiling

        with open(tfile) as f:
            ts = json.load(f)
        kname = kernel_name(dominant, args.prec)
        rec = ts["kernels"].get(kname)
        if ts.get("kernel_source_hash") == profiling.kernel_source_hash(args.prec) and rec:
            traffic = rec["fetch_bytes"] + rec["write_bytes"]

    variants = {}
    if args.prec == "fp64" and not args.no_variants:
        # the FP32 form on the same mesh and state, timed the same way
        g.close()
        g32 = fr.FRMesh(mesh, args.p, mu=mu, flux=args.flux, prec="fp32", ref_rho=1.0, ref_p=p0)
        g32.set_state(U)
        if args.tiles is None:
            g32.autotune(2)
        else:
            g32.set_tiles(*args.tiles)
        for _ in range(args.warmup):
            g32.rk_step(args.dt, args.scheme, 1)
        torch.cuda.synchronize()
        e0.record(stream)
        g32.rk_step(args.dt, args.scheme, args.steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms32 = e0.elapsed_time(e1) / args.steps
        k32 = {k: v for k, v in g32.profile_stages(args.dt, args.scheme, 2).items() if v > 0}
        ab32 = algorithmic_bytes(args.p, "fp32")
        variants["fp32"] = {
            "value": dof * stages / (ms32 * 1e-3), "ms_per_step": ms32, "speedup_vs_fp64": ms_step / ms32,
            "kernel_ms": k32,
            "kernel_gbs": {k: ab32[k] * mesh.n_elem / (k32[k] * 1e-3) / 1e9 for k in k32},
            "finite": bool(np.isfinite(g32.get_state()).all()),
            "dtype": "f32 operators and fluxes, f64 state, RK registers and mass equation"}
        g32.close()

    cpu = None
    if not args.no_cpu:
        try:
            cpu = cpu_baseline(mesh, args.p, U, mu, args.flux)
        except Exception as exc:  # report, never fake
            cpu = {"error": str(exc)}

    wl = (f"TGV Ma0.1 Re1600, {'curved' if not args.affine else 'affine'} periodic {args.n}^3 hex, "
          f"p={args.p}, {args.flux.capitalize()}+BR2, {args.scheme.upper()} dt={args.dt}, "
          f"{'FP64' if args.prec == 'fp64' else 'FP32 operators/fluxes, FP64 state and mass'}")
    out = {
        "metric": "DOF-updates/s per RK stage",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl, "n_elem": mesh.n_elem, "dof": dof, "p": args.p,
                   "tiles": {"elements_per_block": ("256/Ns", "half of 256/Ns")[tiles[0]],
                             "face_block": (256, 128, 64)[tiles[1]],
                             "fused_prepass": fused,
                             "autotune_ms_per_stage": None if tile_ms is None else [float(x) for x in tile_ms]},
                   "stages_per_step": stages, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel_name(dominant, args.prec),
                     "bytes_per_launch": ab[dominant] * mesh.n_elem,
                     "mean_launch_ms": kms[dominant]},
        "stage": {"kernel_ms": kms, "kernel_gbs": gbs, "stage_ms": stage_ms,
                  "stage_min_bytes": stage_bytes,
                  "stage_min_bytes_frac_of_hbm": stage_bytes / (stage_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "variants": variants,
        "cpu_baseline": cpu,
        "setup_s": t_setup,
        "wall_s_timed": t_wall,
        "finite": ok,
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
