"""GPU parity of the low-storage SSP Runge-Kutta scheme and of the body-force source term
against the oracle, through the C ABI, with the FP64 floor rule of the plain residual:
per variable e_v = max|X_gpu - X_ld| / max|X_ld| <= max(1e-12, 2 f_v), f_v the same measure
for the double-precision oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2308_06605_amd import inputs as I

pytestmark = pytest.mark.gpu

MU = 1.0 / 1600.0
G = np.array([0.3, -0.2, 0.1])


def _fr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_06605_amd import fr

    fr.load()
    return fr


def rel(a, b):
    return np.abs(a - b).max(axis=(0, 2)) / np.maximum(np.abs(b).max(axis=(0, 2)), 1e-300)


@pytest.mark.parametrize("nsteps", [1, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ssprk104_steps(nsteps, prec):
    fr = _fr()
    m = I.box_mesh(6, q=2, curve_amp=0.05)
    g = fr.FRMesh(m, 3, mu=MU, flux="roe", prec=prec, ref_rho=1.0, ref_p=1 / (1.4 * 0.01))
    X = g.sol_coords()
    U0 = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=2, amp=0.01)
    g.set_state(U0)
    dt = 2e-3
    g.rk_step(dt, "ssprk104", nsteps)
    Ug = g.get_state()
    g.close()
    Uo = oracle.Oracle(m, 3, mu=MU, flux="roe").rk_step(U0, dt, "ssprk104", nsteps)
    Ul = oracle.Oracle(m, 3, mu=MU, flux="roe", precision="ld").rk_step(U0, dt, "ssprk104", nsteps)
    if prec == "fp64":
        e, f = rel(Ug, Ul), rel(Uo, Ul)
        print(f"ssprk104 x{nsteps} state err {e} floor {f}", flush=True)
        assert np.all(e <= np.maximum(1e-12, 2 * f)), (e, f)
    else:
        # the FP32 form: error relative to the step's increment, at its residual error level
        inc = np.abs(Ul - U0).max(axis=(0, 2))
        e = np.abs(Ug - Ul).max(axis=(0, 2)) / inc
        print(f"ssprk104 fp32 x{nsteps} err/increment {e}", flush=True)
        assert np.all(e < 1e-3), e


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_body_force_residual(flux):
    fr = _fr()
    m = I.box_mesh(5, q=3, curve_amp=0.05, curve_mode="mixed")
    g = fr.FRMesh(m, 3, mu=MU, flux=flux)
    X = g.sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=6, amp=0.02)
    g.set_state(U)
    g.set_body_force(G)
    R = g.residual()
    g.set_body_force(None)
    R0 = g.residual()
    g.close()
    res = {}
    for prec in ("f64", "ld"):
        o = oracle.Oracle(m, 3, mu=MU, flux=flux, precision=prec)
        o.set_body_force(G)
        res[prec] = o.residual(U)
    e, f = rel(R, res["ld"]), rel(res["f64"], res["ld"])
    print(f"{flux} body force err {e} floor {f}", flush=True)
    assert np.all(e <= np.maximum(1e-12, 2 * f)), (e, f)
    assert rel(R, R0)[1:].min() > 1e-3


@pytest.mark.parametrize("scheme", ["lsrk45", "ssprk104", "rk4"])
def test_body_force_uniform_acceleration(scheme):
    """A uniform state under a body force stays uniform, with m and E polynomial in t, which a
    fourth-order scheme integrates exactly; the FP32 form too (its mass equation and state are
    FP64)."""
    fr = _fr()
    m = I.box_mesh(4, q=1)
    for prec in ("fp64", "fp32"):
        g = fr.FRMesh(m, 3, mu=MU, flux="roe", prec=prec, ref_rho=1.0, ref_p=1 / (1.4 * 0.01))
        U0 = I.state_from_coords(g.sol_coords(), I.freestream_state)
        g.set_state(U0)
        g.set_body_force(G)
        dt, n = 2e-3, 10
        g.rk_step(dt, scheme, n)
        U = g.get_state()
        g.close()
        t = dt * n
        rho, m0 = U0[:, 0], U0[:, 1:4]
        exact = U0.copy()
        exact[:, 1:4] = m0 + rho[:, None] * G[None, :, None] * t
        exact[:, 4] = U0[:, 4] + np.einsum("eis,i->es", m0, G) * t + 0.5 * rho * (G @ G) * t * t
        err = np.abs(U - exact).max()
        print(f"{scheme} {prec} uniform acceleration err {err:.3g}", flush=True)
        # FP32 form: the divergence of the uniform O(1) reduced flux rounds to
        # eps32 |D| |F'| 2/h ~ 6e-8 * 11 * 1 * 1.3 ~ 1e-6 per unit time at each point
        assert err < (1e-11 if prec == "fp64" else 1e-6), err
