"""Batches: meshes of different degrees, precisions and closures advanced by one captured HIP
graph per step, the viscous FP32-form meshes by the multi-mesh kernels (one launch per kernel,
stage and degree over all of them) and the others on graph branches of their own.
Every mesh must end bit for bit where fr_rk_step takes an identical mesh alone (each work item
computes what the single-mesh kernel's block does), over several replays with the program's
own eager work and synchronisation between them. Two of the 48-mesh workload's own meshes are
checked against the oracle's step."""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2308_06605_amd import inputs as I

pytestmark = pytest.mark.gpu

MU = 1.0 / 1600.0
P0 = 1.0 / (1.4 * 0.01)


def _fr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_06605_amd import fr

    fr.load()
    return fr


CASES = [  # (n, p, prec, viscous, closure, force)
    (4, 2, "fp64", "br2", None, None),
    (5, 3, "fp32", "br2", None, None),
    (3, 4, "fp64", "ldg", None, (0.1, 0.0, 0.0)),
    (4, 3, "fp64", "br2", "fixed", None),
    (3, 3, "fp64", "br2", "model", None),
    (6, 1, "fp64", "br2", None, None),
    # FP32-form meshes the multi-mesh kernels group by degree, fusion and tiles: several sizes
    # and reference states per degree, a body force, walls, a mesh with the fused pre-pass off and
    # meshes whose tiles differ from their degree's others
    (3, 3, "fp32", "br2", None, (0.0, 0.05, 0.0)),
    (4, 3, "fp32", "br2", "walls", None),
    (3, 2, "fp32", "br2", None, None),
    (5, 2, "fp32", "br2", "nofuse", None),
    (4, 2, "fp32", "br2", None, None),
    (3, 5, "fp32", "br2", None, None),
    (3, 7, "fp32", "br2", None, None),
    (4, 3, "fp32", "br2", "tiles", None),
    (3, 2, "fp32", "br2", "tiles", None),
    # at p = 5 and 6 the second tile choice is two elements per block
    (3, 5, "fp32", "br2", "tiles", None),
    (3, 6, "fp32", "br2", "tiles", None),
]


def _make(fr, case, seed):
    n, p, prec, visc, closure, force = case
    p0 = P0 * (1 + 0.1 * seed)
    if closure == "walls":
        m = I.box_mesh(n, q=2, periodic=(True, False, True), curve_amp=0.04, curve_mode="mixed")
        g = fr.FRMesh(m, p, mu=MU, flux="roe", prec=prec, ref_rho=1.0, ref_p=p0, bc_tag=I.boundary_tags(m),
                      wall_T=1.1 * p0)
    else:
        m = I.box_mesh(n, q=min(max(p, 1), 2), curve_amp=0.04)
        g = fr.FRMesh(m, p, mu=MU, flux="roe", prec=prec, ref_rho=1.0, ref_p=p0, viscous=visc)
    if closure == "nofuse":
        g.set_fusion(False)
    elif closure == "tiles":
        g.set_tiles(1, 2)
    X = g.sol_coords()
    g.set_state(I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=seed, amp=0.02))
    net = None
    if closure == "fixed":
        g.set_eddy_viscosity(np.random.default_rng(seed).uniform(0, 0.002, g.E))
    elif closure == "model":
        F = g.n_features
        net = fr.MLP(F, M.init_params(F, seed), np.full(F, -5.0), np.full(F, 5.0))
        g.set_sgs_model(net, nu_scale=1e-3)
    if force is not None:
        g.set_body_force(force)
    return g, net


@pytest.mark.parametrize("scheme,multi", [("lsrk45", True), ("ssprk104", True), ("rk4", True), ("lsrk45", False)])
def test_batch_matches_single_meshes(scheme, multi):
    import torch

    fr = _fr()
    dts = [1e-3 * (1 + 0.1 * i) for i in range(len(CASES))]
    batch_meshes, single_meshes, nets = [], [], []
    for i, c in enumerate(CASES):
        g, net = _make(fr, c, seed=i)
        batch_meshes.append(g)
        nets.append(net)
        g2, net2 = _make(fr, c, seed=i)
        single_meshes.append(g2)
        nets.append(net2)
    b = fr.Batch(batch_meshes, dts, scheme, multi=multi)
    # 2 steps: the one-step graph twice; 9: the chained 8-step graph, then the one-step graph
    for rep, nsteps in enumerate((2, 9, 2)):
        b.step(nsteps)
        torch.cuda.synchronize()
        for g2, dt in zip(single_meshes, dts):
            g2.rk_step(dt, scheme, nsteps)
        torch.cuda.synchronize()
        for i, (g, g2) in enumerate(zip(batch_meshes, single_meshes)):
            Ub, Us = g.get_state(), g2.get_state()
            assert np.isfinite(Ub).all()
            assert np.array_equal(Ub, Us), (rep, i, np.abs(Ub - Us).max())
        # eager work on the batch's meshes between replays: a residual and a state round trip
        for g in batch_meshes:
            g.residual()
            g.set_state(g.get_state())
    b.close()
    for g in batch_meshes + single_meshes:
        g.close()
    for net in nets:
        if net is not None:
            net.close()


def test_many_meshes_in_one_group():
    """33 FP32-form meshes of one degree and one tile setting, of 27 to 80 elements in uneven
    order: one multi-mesh group whose launches cover all of them, so a block's mesh is found by
    bisection over 33 prefix sums. Every mesh ends bit for bit where fr_rk_step takes it."""
    import torch

    fr = _fr()
    rng = np.random.default_rng(5)
    shapes = [tuple(int(x) for x in rng.integers(3, 6, 3)) for _ in range(33)]
    meshes, singles, dts = [], [], []
    for i, sh in enumerate(shapes):
        m = I.box_mesh(sh, q=2, curve_amp=0.03)
        p0 = P0 * (1 + 0.01 * i)
        gs = []
        for _ in range(2):
            g = fr.FRMesh(m, 2, mu=MU, flux="roe", prec="fp32", ref_rho=1.0, ref_p=p0)
            X = g.sol_coords()
            g.set_state(I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=i, amp=0.02))
            gs.append(g)
        meshes.append(gs[0])
        singles.append(gs[1])
        dts.append(5e-4 * (1 + 0.02 * i))
    b = fr.Batch(meshes, dts, "lsrk45")
    for rep, nsteps in enumerate((2, 8)):
        b.step(nsteps)
        torch.cuda.synchronize()
        for g, dt in zip(singles, dts):
            g.rk_step(dt, "lsrk45", nsteps)
        for i, (g, g2) in enumerate(zip(meshes, singles)):
            Ub, Us = g.get_state(), g2.get_state()
            assert np.isfinite(Ub).all()
            assert np.array_equal(Ub, Us), (rep, i, shapes[i])
    b.close()
    for g in meshes + singles:
        g.close()


def test_batch_errors():
    fr = _fr()
    g, _ = _make(fr, CASES[0], 0)
    with pytest.raises(fr.FRError):
        fr.Batch([g, g], [1e-3, 1e-3])
    with pytest.raises(fr.FRError):
        fr.Batch([g], [0.0])
    g.close()


def test_workload_meshes_against_the_oracle():
    """Two of the 48-mesh workload's own meshes (the smallest of degree 2 and of degree 4 or 5:
    walled channels, FP32 form, their own Mach number and step size) advanced one LSRK45 step by
    the batch, against the oracle's step in long double; errors relative to the step's increment
    per variable."""
    import torch

    import oracle
    from paper_2308_06605_amd import batched as B

    fr = _fr()
    by_cost = sorted(B.workload(48, 0), key=lambda s: s["n"] ** 3 * (s["p"] + 1) ** 3)
    specs = [next(s for s in by_cost if s["p"] == 2), next(s for s in by_cost if s["p"] >= 4)]
    meshes, states, dts = [], [], []
    for spec in specs:
        g, U = B.build(fr, spec, walls=True, prec="fp32")
        meshes.append(g)
        states.append(U)
        dts.append(B.stable_dt(spec["n"], spec["p"], spec["mach"]))
    b = fr.Batch(meshes, dts, "lsrk45")
    b.step(1)
    torch.cuda.synchronize()
    for spec, g, U0, dt in zip(specs, meshes, states, dts):
        Ug = g.get_state()
        m = I.box_mesh(spec["n"], q=1, periodic=(True, False, True))
        p0 = 1.0 / (1.4 * spec["mach"] ** 2)
        Ul = oracle.Oracle(m, spec["p"], mu=B.MU, flux="roe", precision="ld", bc_tag=I.boundary_tags(m),
                           wall_T=p0).rk_step(U0, dt, "lsrk45", 1)
        inc = np.abs(Ul - U0).max(axis=(0, 2))
        e = np.abs(Ug - Ul).max(axis=(0, 2)) / inc
        print(f"workload mesh n={spec['n']} p={spec['p']} Mach {spec['mach']:.3f}: step error / increment {e}",
              flush=True)
        assert np.all(e < 5e-3), e
    b.close()
    for g in meshes:
        g.close()
