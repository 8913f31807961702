"""GPU tests of the FP32 form (FP32 operators and fluxes, FP64 state, RK registers and mass
equation, reference-state split of the pressure and enthalpy).

The error against the long-double oracle is stated per variable (max-norm, relative to the
variable's maximum) and jointly (L2 over all variables), and bounded here at the levels
measured on MI355X with margin:
  8^3 p=3 TGV:  joint L2 ~1.1e-5, per variable <= 1e-4 (momentum)
  16^3 p=3 TGV: joint L2 ~5e-5,  per variable <= 2.4e-4
  4^3 p=4..7 perturbed TGV: joint L2 <= 1.2e-6, per variable <= 2.2e-4
This is the FP32 round-off of O(1) fluxes differentiated at 2/h: 1e-5 per variable is below
the FP32 floor of this Mach 0.1 workload. The split is what makes it usable at all: demoting
the state as it is (the float oracle) is off by 0.4 % to 2 %.
"""
import numpy as np
import pytest

import oracle
from paper_2308_06605_amd import inputs as I

pytestmark = pytest.mark.gpu

P0 = 1.0 / (1.4 * 0.01)
MU = 1.0 / 1600.0


def _fr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_06605_amd import fr

    fr.load()
    return fr


def errors(R, Rl):
    e = np.abs(R - Rl).max(axis=(0, 2)) / np.abs(Rl).max(axis=(0, 2))
    joint = np.sqrt(((R - Rl) ** 2).sum() / (Rl ** 2).sum())
    return e, joint


@pytest.mark.parametrize("n,bound_var,bound_joint", [(8, 3e-4, 4e-5), (16, 8e-4, 2e-4)])
def test_fp32_residual_error(n, bound_var, bound_joint):
    fr = _fr()
    p = 3
    m = I.box_mesh(n, q=3, curve_amp=0.05)
    g = fr.FRMesh(m, p, mu=MU, flux="roe", prec="fp32", ref_rho=1.0, ref_p=P0)
    U = I.state_from_coords(g.sol_coords(), I.tgv_state)
    g.set_state(U)
    R = g.residual()
    g.close()
    Rl = oracle.Oracle(m, p, mu=MU, flux="roe", precision="ld").residual(U)
    e, joint = errors(R, Rl)
    Rf = oracle.Oracle(m, p, mu=MU, flux="roe", precision="f32").residual(U)
    _, joint_naive = errors(Rf, Rl)
    print(f"{n}^3 fp32 form: per-variable {e} joint L2 {joint:.3g}; naive float {joint_naive:.3g}", flush=True)
    assert np.all(e < bound_var), e
    assert joint < bound_joint, joint
    assert joint < joint_naive / 50


@pytest.mark.parametrize("p", [4, 5, 6, 7])
def test_fp32_residual_error_high_degree(p):
    """The FP32 form at p = 4..7 on a small curved (isoparametric) mesh with a perturbed TGV,
    every element against the long-double oracle; both the separate and the fused kernels (the
    single-pass tail up to p = 6, the rounds at p = 7) produce this residual's face data in an
    RK run, and fused stepping is bitwise the separate one (test_gpu_fused_prepass), so the
    residual checks the arithmetic of both."""
    fr = _fr()
    m = I.box_mesh(4, q=p, curve_amp=0.05)
    g = fr.FRMesh(m, p, mu=MU, flux="roe", prec="fp32", ref_rho=1.0, ref_p=P0)
    X = g.sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=p, amp=0.01)
    g.set_state(U)
    R = g.residual()
    g.close()
    Rl = oracle.Oracle(m, p, mu=MU, flux="roe", precision="ld").residual(U)
    e, joint = errors(R, Rl)
    Rf = oracle.Oracle(m, p, mu=MU, flux="roe", precision="f32").residual(U)
    _, joint_naive = errors(Rf, Rl)
    print(f"4^3 p={p} fp32 form: per-variable {e} joint L2 {joint:.3g}; naive float {joint_naive:.3g}", flush=True)
    # measured on MI355X: per variable <= 2.2e-4 (momentum, p = 7), joint L2 <= 1.2e-6; the
    # mass residual's error (1e-6 to 5e-6 of its maximum) is the Roe dissipation's, which is
    # formed in FP32 like the other interface terms
    assert np.all(e < 6e-4), e
    assert joint < 4e-6, joint
    assert joint < joint_naive / 50


def test_fp32_conservation():
    fr = _fr()
    p = 3
    m = I.box_mesh(4, q=3, curve_amp=0.05, curve_mode="mixed")
    g = fr.FRMesh(m, p, mu=MU, flux="roe", prec="fp32", ref_rho=1.0, ref_p=P0)
    X = g.sol_coords()
    g.set_state(I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=3, amp=0.01))
    R = g.residual()
    _, dJ, _, _ = oracle.Oracle(m, p).geometry()
    w = np.polynomial.legendre.leggauss(p + 1)[1]
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    tot = np.einsum("evs,es,s->v", R, dJ, W)
    mag = np.einsum("evs,es,s->v", np.abs(R), dJ, W)
    rel = np.abs(tot) / mag
    assert rel[0] < 1e-12, rel  # the mass equation is FP64
    assert np.all(rel[1:] < 1e-5), rel


def test_fp32_kinetic_energy_dissipation():
    """BR2 TGV at Re 1600 on 16^3 p=3 to t = 2: the dissipation rate -dE_k/dt of the FP32 form
    stays within 1 % of the FP64 run's (relative to its maximum over the run)."""
    fr = _fr()
    p, dt, nsteps, every = 3, 1e-3, 2000, 250
    m = I.box_mesh(16, q=1)
    eps = {}
    for prec in ("fp64", "fp32"):
        g = fr.FRMesh(m, p, mu=MU, flux="roe", prec=prec, ref_rho=1.0, ref_p=P0)
        g.set_state(I.state_from_coords(g.sol_coords(), I.tgv_state))
        vals = []
        for k in range(nsteps // every + 1):
            vals.append(-g.kinetic_energy()[1])
            if k < nsteps // every:
                g.rk_step(dt, "lsrk45", every)
        g.close()
        eps[prec] = np.array(vals)
    ref = np.abs(eps["fp64"]).max()
    err = np.abs(eps["fp32"] - eps["fp64"]).max() / ref
    print("dissipation rate fp64", eps["fp64"], "fp32", eps["fp32"], "max rel err", err, flush=True)
    assert np.all(eps["fp64"] > 0)
    assert err < 0.01, err


def test_kinetic_energy_diagnostic_matches_oracle():
    """E_k and dE_k/dt from the library's reduction against the same quadrature done here with
    the oracle's residual and geometry."""
    fr = _fr()
    p = 3
    m = I.box_mesh(6, q=3, curve_amp=0.05)
    g = fr.FRMesh(m, p, mu=MU, flux="roe")
    U = I.state_from_coords(g.sol_coords(), I.tgv_state)
    g.set_state(U)
    ek, dek = g.kinetic_energy()
    o = oracle.Oracle(m, p, mu=MU, flux="roe")
    R = o.residual(U)
    _, dJ, _, _ = o.geometry()
    w = np.polynomial.legendre.leggauss(p + 1)[1]
    W = np.einsum("k,j,i->kji", w, w, w).ravel() * dJ
    rho, mom = U[:, 0], U[:, 1:4]
    q2 = (mom ** 2).sum(axis=1) / rho ** 2
    ek_ref = (W * 0.5 * rho * q2).sum() / W.sum()
    dek_ref = (W * ((mom * R[:, 1:4]).sum(axis=1) / rho - 0.5 * q2 * R[:, 0])).sum() / W.sum()
    assert abs(ek - ek_ref) < 1e-13 * abs(ek_ref)
    assert abs(dek - dek_ref) < 1e-9 * abs(ek_ref)
