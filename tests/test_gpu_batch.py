"""Batches: meshes of different degrees, precisions and closures advanced by one captured HIP
graph per step. Every mesh must end bit for bit where fr_rk_step takes an identical mesh alone
(the same kernels in the same order within each mesh), over several replays with the
program's own eager work and synchronisation between them."""
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
]


def _make(fr, case, seed):
    n, p, prec, visc, closure, force = case
    m = I.box_mesh(n, q=min(max(p, 1), 2), curve_amp=0.04)
    g = fr.FRMesh(m, p, mu=MU, flux="roe", prec=prec, ref_rho=1.0, ref_p=P0, viscous=visc)
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


@pytest.mark.parametrize("scheme", ["lsrk45", "ssprk104", "rk4"])
def test_batch_matches_single_meshes(scheme):
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
    b = fr.Batch(batch_meshes, dts, scheme)
    for rep in range(3):
        b.step(2)
        torch.cuda.synchronize()
        for g2, dt in zip(single_meshes, dts):
            g2.rk_step(dt, scheme, 2)
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


def test_batch_errors():
    fr = _fr()
    g, _ = _make(fr, CASES[0], 0)
    with pytest.raises(fr.FRError):
        fr.Batch([g, g], [1e-3, 1e-3])
    with pytest.raises(fr.FRError):
        fr.Batch([g], [0.0])
    g.close()
