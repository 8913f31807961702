"""Many uneven meshes advanced together: the batched workload and its throughput measurement.

Workload (seeded with numpy.random.default_rng(seed)): n_mesh channel meshes on [0, 2 pi)^3,
periodic in x and z with isothermal no-slip walls in y at the flow's temperature, element counts
drawn log-uniformly from [8^3, 40^3] (n = round(cbrt(N)) elements per direction), degree p
uniform in {2, 3, 4, 5}, a uniform flow along x at Mach 0.2 to 0.5 (|u| = 1) with a seeded
smooth random perturbation, Roe + BR2 at mu = 1e-4, the FP32 form (FP32 operators and fluxes,
FP64 state and mass equation) and LSRK45 with dt from the stability estimate
dt = 1.5 h / ((|u| + c)(p + 1)(p + 2) 1.7). Each mesh's tile shapes come from the autotuner
(fr_autotune) before anything is timed. --periodic makes fully periodic boxes instead (the flow
direction is then (1, 0.5, 0.25) normalised), --fp64 runs the FP64 kernels, --no-autotune keeps the
default tiles.

Three ways to run the same steps are timed on the same meshes and state:
  sequential  fr_rk_step on each mesh in turn (11 to 15 kernel launches per mesh and step),
  branches    captured HIP graphs (of one step and of 8 chained steps), every mesh on a graph
              branch of its own,
  multi       the same graphs, in which each degree's meshes are stepped by the
              multi-mesh kernels: per stage one face and one volume launch covering all of them,
              block b of a launch being some mesh's element or face block (fr_batch_create).
Throughput is the total DOF-updates per second per RK stage; the roofline fraction is the
meshes' summed two-pass minimum bytes per stage over the stage time at 8 TB/s.

  python -m paper_2308_06605_amd.batched [--n-mesh 48] [--steps 10] [--seed 0] [--sizes 8 40]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import inputs as I
from .profiling import algorithmic_bytes

GAMMA = 1.4
MU = 1e-4


def workload(n_mesh: int, seed: int, n_min: int = 8, n_max: int = 40):
    rng = np.random.default_rng(seed)
    N = np.exp(rng.uniform(math.log(n_min ** 3), math.log(n_max ** 3), n_mesh))
    n = np.maximum(3, np.rint(np.cbrt(N)).astype(int))
    p = rng.integers(2, 6, n_mesh)
    mach = rng.uniform(0.2, 0.5, n_mesh)
    return [dict(n=int(n[i]), p=int(p[i]), mach=float(mach[i]), seed=seed * 1000 + i) for i in range(n_mesh)]


def stable_dt(n: int, p: int, mach: float) -> float:
    h = 2 * math.pi / n
    c = 1.0 / mach
    return 1.5 * h / ((1.0 + c) * (p + 1) * (p + 2) * 1.7)


def build(fr, spec, walls=True, prec="fp32"):
    p0 = 1.0 / (GAMMA * spec["mach"] ** 2)
    kw = dict(prec="fp32", ref_rho=1.0, ref_p=p0) if prec == "fp32" else {}
    if walls:
        m = I.box_mesh(spec["n"], q=1, periodic=(True, False, True))
        g = fr.FRMesh(m, spec["p"], mu=MU, flux="roe", bc_tag=I.boundary_tags(m), wall_T=p0, **kw)
        X = g.sol_coords()
        U = I.state_from_coords(X, I.freestream_state, mach=spec["mach"], direction=(1.0, 0.0, 0.0))
    else:
        m = I.box_mesh(spec["n"], q=1)
        g = fr.FRMesh(m, spec["p"], mu=MU, flux="roe", **kw)
        X = g.sol_coords()
        U = I.state_from_coords(X, I.freestream_state, mach=spec["mach"])
    U += I.random_smooth_perturbation(X, seed=spec["seed"], amp=0.01)
    g.set_state(U)
    return g, U


def run(n_mesh=48, steps=16, warmup=2, seed=0, walls=True, prec="fp32", autotune=True, sizes=(8, 40)):
    import torch

    from . import fr

    fr.load()
    specs = workload(n_mesh, seed, *sizes)
    t0 = time.time()
    meshes, states, dts = [], [], []
    for s in specs:
        g, U = build(fr, s, walls, prec)
        meshes.append(g)
        states.append(U)
        dts.append(stable_dt(s["n"], s["p"], s["mach"]))
    setup_s = time.time() - t0
    t0 = time.time()
    tiles = [g.autotune(3)[0] if autotune else g.tiles() for g in meshes]
    fused = [g.fusion() for g in meshes]
    autotune_s = time.time() - t0
    dof = sum(g.E * g.Ns for g in meshes)
    stages = 5
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def reset():
        for g, U in zip(meshes, states):
            g.set_state(U)
        torch.cuda.synchronize()

    # sequential
    for g, dt in zip(meshes, dts):
        g.rk_step(dt, "lsrk45", warmup)
    reset()
    e0.record(stream)
    for _ in range(steps):
        for g, dt in zip(meshes, dts):
            g.rk_step(dt, "lsrk45", 1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_seq = e0.elapsed_time(e1) / steps
    U_seq = [g.get_state() for g in meshes]
    # the two captured forms
    timed = {}
    same = True
    for name, multi in (("branches", False), ("multi", True)):
        reset()
        t1 = time.time()
        b = fr.Batch(meshes, dts, "lsrk45", multi=multi)
        capture_s = time.time() - t1
        b.step(warmup)
        reset()
        e0.record(stream)
        b.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        same = same and all(np.array_equal(g.get_state(), u) for g, u in zip(meshes, U_seq))
        b.close()
        timed[name] = {"ms_per_step": ms, "dof_updates_per_s": dof * stages / (ms * 1e-3), "capture_s": capture_s}
    finite = all(np.isfinite(u).all() for u in U_seq)
    for g in meshes:
        g.close()
    # the two-pass minimum bytes per stage of every mesh
    stage_bytes = sum(algorithmic_bytes(s["p"], prec)["stage_min"] * s["n"] ** 3 for s in specs)
    for rec in [timed["branches"], timed["multi"]]:
        rec["roofline_frac"] = stage_bytes / (rec["ms_per_step"] / stages * 1e-3) / 8e12
    geo = "channel meshes (isothermal walls in y)" if walls else "periodic box meshes"
    out = {
        "workload": f"{n_mesh} {geo}, log-uniform {sizes[0]}^3..{sizes[1]}^3 elements, p in 2..5, Mach 0.2-0.5, "
                    f"Roe+BR2 mu={MU}, {'FP32 form' if prec == 'fp32' else 'FP64'}, LSRK45, "
                    f"{'autotuned' if autotune else 'default'} tiles, seed {seed}",
        "n_mesh": n_mesh, "dof": int(dof), "elements": int(sum(g.E for g in meshes)),
        "steps": steps, "stages_per_step": stages,
        "sequential": {"ms_per_step": ms_seq, "dof_updates_per_s": dof * stages / (ms_seq * 1e-3),
                       "roofline_frac": stage_bytes / (ms_seq / stages * 1e-3) / 8e12},
        "batch_branches": timed["branches"], "batch_multi": timed["multi"],
        "stage_min_bytes": stage_bytes,
        "speedup_multi_vs_sequential": ms_seq / timed["multi"]["ms_per_step"],
        "speedup_multi_vs_branches": timed["branches"]["ms_per_step"] / timed["multi"]["ms_per_step"],
        "bitwise_equal": bool(same), "finite": bool(finite),
        "setup_s": setup_s, "autotune_s": autotune_s,
        "tiles_chosen": {f"{e},{f}": sum(1 for t in tiles if tuple(t) == (e, f)) for e in (0, 1) for f in (0, 1, 2)},
        "fused_prepass": sum(fused),
        "multi_groups": len({(s["p"], fz, tuple(t)) for s, t, fz in zip(specs, tiles, fused)}),
        "meshes": [dict(s, dt=dt, tiles=list(t), fused=fz) for s, dt, t, fz in zip(specs, dts, tiles, fused)],
    }
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2308_06605_amd.batched")
    ap.add_argument("--n-mesh", type=int, default=48)
    ap.add_argument("--steps", type=int, default=16, help="timed steps (fr_batch_step: 8-step replays first)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--periodic", action="store_true", help="fully periodic boxes instead of channels")
    ap.add_argument("--fp64", action="store_true", help="the FP64 kernels instead of the FP32 form")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tiles")
    ap.add_argument("--sizes", type=int, nargs=2, default=(8, 40), metavar=("MIN", "MAX"),
                    help="elements per direction: the meshes' element counts are log-uniform in MIN^3..MAX^3")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = run(a.n_mesh, a.steps, a.warmup, a.seed, not a.periodic, "fp64" if a.fp64 else "fp32",
              not a.no_autotune, tuple(a.sizes))
    line = {k: v for k, v in res.items() if k != "meshes"}
    print(json.dumps(line), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
