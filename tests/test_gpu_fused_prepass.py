"""The volume kernel's fused pre-pass of the next stage (both precisions).

Within one fr_rk_step call every stage after the first takes its face values and broken
gradient from the previous stage's volume kernel (k_volume with the pre-pass tail); the first
stage of a call runs the stand-alone k_prepass. The two compute the same sums in the same
order, so n steps in one call must equal n calls of one step bit for bit: the step boundaries
of the second run go through k_prepass, those of the first through the fused tail. The
parametrisation covers every tail variant: BR2 (values and gradient, in one pass up to p = 5
in FP64 and p = 6 in FP32, in chunks of variables above), LDG and the Euler equations (values
only), the closure, walls, and the three Runge-Kutta schemes (each hands a different register
to the next stage).
"""
import numpy as np
import pytest

from paper_2308_06605_amd import inputs as I

pytestmark = pytest.mark.gpu


def _fr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_06605_amd import fr

    fr.load()
    return fr


CASES = [
    # p, scheme, mu, viscous, extra
    (3, "lsrk45", 1e-3, "br2", None),
    (3, "rk4", 1e-3, "br2", None),
    (0, "lsrk45", 1e-3, "br2", None),
    (1, "rk4", 1e-3, "br2", None),
    (1, "lsrk45", 1e-3, "br2", "fp32"),
    (2, "ssprk104", 1e-3, "br2", None),
    (4, "rk4", 1e-3, "br2", None),
    (5, "lsrk45", 1e-3, "br2", None),
    (6, "ssprk104", 1e-3, "br2", None),
    (7, "rk4", 1e-3, "br2", None),
    (4, "lsrk45", 1e-3, "ldg", None),
    (3, "lsrk45", 0.0, "br2", None),
    (3, "lsrk45", 1e-3, "br2", "closure"),
    (3, "rk4", 1e-3, "br2", "walls"),
    (3, "lsrk45", 1e-3, "br2", "fp32"),
    (7, "rk4", 1e-3, "br2", "fp32"),
    (4, "ssprk104", 0.0, "br2", "fp32"),
    (4, "lsrk45", 1e-3, "br2", "fp32"),
    (5, "rk4", 1e-3, "br2", "fp32"),
    (6, "lsrk45", 1e-3, "br2", "fp32"),
    (2, "lsrk45", 1e-3, "br2", "fp32 walls"),
    # 75 elements: a ragged last block at every tile choice of p = 3 (4 or 2 elements per block)
    (3, "lsrk45", 1e-3, "br2", "ragged"),
    (3, "rk4", 1e-3, "br2", "fp32 ragged"),
]


@pytest.mark.parametrize("p,scheme,mu,viscous,extra", CASES)
def test_steps_in_one_call_equal_separate_calls(p, scheme, mu, viscous, extra):
    fr = _fr()
    p0 = 1.0 / (1.4 * 0.01)
    if extra is not None and "walls" in extra:
        m = I.box_mesh((4, 5, 4), q=2, periodic=(True, False, True), curve_amp=0.02, curve_mode="mixed")
        kw = dict(bc_tag=I.boundary_tags(m), wall_T=p0)
    elif extra is not None and "ragged" in extra:
        m = I.box_mesh((5, 5, 3), q=max(1, min(p, 3)), curve_amp=0.04)
        kw = {}
    else:
        m = I.box_mesh(4, q=max(1, min(p, 3)), curve_amp=0.04)
        kw = {}
    if extra is not None and "fp32" in extra:
        kw.update(prec="fp32", ref_rho=1.0, ref_p=p0)
    g = fr.FRMesh(m, p, mu=mu, flux="roe", viscous=viscous, **kw)
    X = g.sol_coords()
    U0 = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=p, amp=0.01)
    if extra == "closure":
        g.set_eddy_viscosity(np.random.default_rng(1).uniform(0, 2e-3, m.n_elem))
    dt, n = 2e-4, 3
    tiles = [(0, 0), (1, 1)] if extra is not None and "ragged" in extra else [g.tiles()]
    for epb, fbs in tiles:
        g.set_tiles(epb, fbs)
        g.set_state(U0)
        g.rk_step(dt, scheme, n)
        A = g.get_state()
        g.set_state(U0)
        for _ in range(n):
            g.rk_step(dt, scheme, 1)
        B = g.get_state()
        assert np.isfinite(A).all()
        assert not np.array_equal(A, U0)
        assert np.array_equal(A, B), (epb, fbs, np.abs(A - B).max())
    g.close()
