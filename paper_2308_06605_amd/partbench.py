"""What the partitioned run costs on one GPU: a mesh stepped whole and split into parts that
exchange their shared faces once per stage (fr_part_*), and the exchange's own messages.

The parts run one after another on one stream here, so the split's step time is the unsplit
kernels' work plus the exchange (pack and unpack kernels) plus the smaller launches; the
message bytes per stage are what several GPUs would send each other over xGMI.

  python -m paper_2308_06605_amd.partbench [--n 64] [--p 3] [--blocks 2 2 2] [--steps 10]

Blocks: the box is cut into bx * by * bz boxes of elements, part index bx-fastest.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import inputs as I

MU = 1.0 / 1600.0
P0 = 1.0 / (1.4 * 0.01)
LINK_GBS = 153.0  # one xGMI link, per direction (vendor figure)


def block_map(n: int, blocks) -> np.ndarray:
    """Element -> part for an n^3 box (element ie + n (je + n ke)) cut into blocks[0..2] boxes."""
    e = np.arange(n ** 3)
    ie, je, ke = e % n, (e // n) % n, e // (n * n)
    bx, by, bz = blocks
    return ((ie * bx // n) + bx * ((je * by // n) + by * (ke * bz // n))).astype(np.int32)


def run(n=64, p=3, blocks=(2, 2, 2), steps=10, prec="fp64"):
    import torch

    from . import fr

    torch.cuda.set_device(0)
    m = I.box_mesh(n, q=p, curve_amp=0.05)
    kw = dict(mu=MU, flux="roe")
    if prec == "fp32":
        kw.update(prec="fp32", ref_rho=1.0, ref_p=P0)
    g = fr.FRMesh(m, p, **kw)
    U = I.state_from_coords(g.sol_coords(), I.tgv_state)
    g.set_state(U)
    tiles, _ = g.autotune(2)
    fused = g.fusion()
    g.set_state(U)
    part = block_map(n, blocks)
    grp = fr.PartitionGroup(m, p, part, **kw)
    for pm in grp.parts:
        pm.set_tiles(*tiles)
        pm.set_fusion(fused)
    grp.set_state(U)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(step):
        step(1)
        torch.cuda.synchronize()
        e0.record(stream)
        step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_whole = timed(lambda k: g.rk_step(2.5e-4, "lsrk45", k))
    ms_split = timed(lambda k: grp.rk_step(2.5e-4, "lsrk45", k))
    same = np.array_equal(g.get_state(), grp.get_state())
    # the exchange alone: every ordered pair's pack and unpack, as one stage does them
    pairs = [(q, r) for q in range(grp.n_part) for r in range(grp.n_part) if q != r and grp.halo_size(q, r)[0] > 0]
    bufs = {(q, r): torch.empty(grp.halo_size(q, r)[1] // 8 + 1, dtype=torch.float64, device="cuda")
            for q, r in pairs}

    def exchange(k):
        for _ in range(k):
            for q, r in pairs:
                grp.halo_pack(q, r, bufs[(q, r)])
            for q, r in pairs:
                grp.halo_unpack(r, q, bufs[(q, r)])

    ms_exchange = timed(exchange)
    msg = {f"{q}->{r}": grp.halo_size(q, r)[1] for q, r in pairs}
    stages = 5
    per_part = max(sum(b for (q, r), b in zip(pairs, msg.values()) if q == s) for s in range(grp.n_part))
    g.close()
    grp.close()
    dof = n ** 3 * (p + 1) ** 3
    return {
        "workload": f"TGV curved {n}^3 p={p} {prec.upper()}, LSRK45, {blocks[0]}x{blocks[1]}x{blocks[2]} parts",
        "ms_per_step_whole": ms_whole, "ms_per_step_split": ms_split,
        "split_overhead": ms_split / ms_whole - 1.0,
        "ms_exchange_per_stage": ms_exchange, "exchange_share_of_split_stage": ms_exchange / (ms_split / stages),
        "bitwise_equal": bool(same), "message_bytes": msg, "pairs": len(pairs),
        "max_bytes_sent_per_part_per_stage": per_part,
        "xgmi_us_per_stage_at_one_link": per_part / (LINK_GBS * 1e9) * 1e6,
        "whole_dof_updates_per_s": dof * stages / (ms_whole * 1e-3),
        "tiles": list(tiles), "fused_prepass": bool(fused),
    }


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2308_06605_amd.partbench")
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--blocks", type=int, nargs=3, default=(2, 2, 2))
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--prec", choices=("fp64", "fp32"), default="fp64")
    a = ap.parse_args(argv)
    print(json.dumps(run(a.n, a.p, tuple(a.blocks), a.steps, a.prec)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
