"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, element by element.

Floating-point gate (double precision): per variable v, e_v = max|R_gpu - R_ld| / max|R_ld|
against the long-double oracle must satisfy e_v <= max(1e-12, 2 f_v), where f_v is the same
measure for the double-precision oracle. f_v is the round-off floor that any two correct FP64
implementations share on that workload (the low-Mach fluxes are large against their
divergence); it is measured in the same test.
"""
import numpy as np
import pytest

import oracle
from paper_2308_06605_amd import inputs as I

pytestmark = pytest.mark.gpu


def _fr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_06605_amd import fr

    fr.load()
    return fr


def rel(a, b):
    return np.abs(a - b).max(axis=(0, 2)) / np.maximum(np.abs(b).max(axis=(0, 2)), 1e-300)


def check_residual(mesh, p, U, **kw):
    fr = _fr()
    g = fr.FRMesh(mesh, p, **kw)
    g.set_state(U)
    R = g.residual()
    g.close()
    okw = {k: v for k, v in kw.items() if k in ("mu", "flux", "eta", "gamma", "prandtl")}
    Ro = oracle.Oracle(mesh, p, **okw).residual(U)
    Rl = oracle.Oracle(mesh, p, precision="ld", **okw).residual(U)
    e, f = rel(R, Rl), rel(Ro, Rl)
    print(f"p={p} E={mesh.n_elem} kw={kw} gpu err {e} oracle floor {f}", flush=True)
    assert np.all(e <= np.maximum(1e-12, 2 * f)), (e, f)
    return R, Rl


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_tgv_8cubed_p3_viscous(flux):
    m = I.box_mesh(8, q=1)
    fr = _fr()
    X = fr.FRMesh(m, 3).sol_coords()
    U = I.state_from_coords(X, I.tgv_state)
    check_residual(m, 3, U, mu=1 / 1600, flux=flux)


def test_vortex_euler():
    m = I.box_mesh((8, 8, 3), lo=(-5, -5, -1), hi=(5, 5, 1), q=1)
    fr = _fr()
    U = I.state_from_coords(fr.FRMesh(m, 3).sol_coords(), I.vortex_state)
    check_residual(m, 3, U, flux="rusanov")


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5, 6, 7])
def test_all_orders_curved_scrambled(p):
    q = max(p, 1)
    m = I.box_mesh(3, q=q, curve_amp=0.05 if p > 0 else 0.0, curve_mode="mixed")
    m, _ = I.scramble_mesh(m, seed=p)
    fr = _fr()
    X = fr.FRMesh(m, p).sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=p, amp=0.02)
    check_residual(m, p, U, mu=0.01, flux="roe")
    check_residual(m, p, U, mu=0.0, flux="rusanov")


def test_freestream_curved_gpu():
    fr = _fr()
    m = I.box_mesh(4, q=3, curve_amp=0.05, curve_mode="mixed")
    g = fr.FRMesh(m, 3, mu=1 / 1600, flux="roe")
    g.set_state(I.state_from_coords(g.sol_coords(), I.freestream_state))
    assert np.abs(g.residual()).max() < 1e-9


def test_conservation_gpu():
    fr = _fr()
    p = 3
    m = I.box_mesh(4, q=3, curve_amp=0.05, curve_mode="mixed")
    g = fr.FRMesh(m, p, mu=1 / 1600, flux="roe")
    X = g.sol_coords()
    g.set_state(I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=3, amp=0.01))
    R = g.residual()
    _, dJ, _, _ = oracle.Oracle(m, p).geometry()
    w = np.polynomial.legendre.leggauss(p + 1)[1]
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    tot = np.einsum("evs,es,s->v", R, dJ, W)
    mag = np.einsum("evs,es,s->v", np.abs(R), dJ, W)
    assert np.all(np.abs(tot) / mag < 1e-12), tot / mag


@pytest.mark.parametrize("scheme,nsteps", [("rk4", 10), ("lsrk45", 4)])
def test_rk_steps_8cubed(scheme, nsteps):
    fr = _fr()
    m = I.box_mesh(8, q=1)
    g = fr.FRMesh(m, 3, mu=1 / 1600, flux="rusanov")
    U0 = I.state_from_coords(g.sol_coords(), I.tgv_state)
    g.set_state(U0)
    g.rk_step(1e-3, scheme, nsteps)
    Ug = g.get_state()
    Uo = oracle.Oracle(m, 3, mu=1 / 1600).rk_step(U0, 1e-3, scheme, nsteps)
    Ul = oracle.Oracle(m, 3, mu=1 / 1600, precision="ld").rk_step(U0, 1e-3, scheme, nsteps)
    e = rel(Ug, Ul)
    f = rel(Uo, Ul)
    print(scheme, "state err", e, "floor", f, flush=True)
    assert np.all(e <= np.maximum(1e-12, 2 * f)), (e, f)


def test_determinism_and_restart():
    fr = _fr()
    m = I.box_mesh(4, q=2, curve_amp=0.05)
    g = fr.FRMesh(m, 3, mu=1 / 1600, flux="roe")
    U0 = I.state_from_coords(g.sol_coords(), I.tgv_state)
    g.set_state(U0)
    R1 = g.residual()
    R2 = g.residual()
    assert np.array_equal(R1, R2)
    g.rk_step(1e-3, "lsrk45", 4)
    U4 = g.get_state()
    g.set_state(U0)
    g.rk_step(1e-3, "lsrk45", 2)
    Uh = g.get_state()
    g.set_state(Uh)  # checkpoint / restart
    g.rk_step(1e-3, "lsrk45", 2)
    assert np.array_equal(g.get_state(), U4)


def test_nonfinite_detection():
    fr = _fr()
    m = I.box_mesh(3, q=1)
    g = fr.FRMesh(m, 2, mu=0.01, check_finite=True)
    U = I.state_from_coords(g.sol_coords(), I.tgv_state)
    g.set_state(U)
    g.residual()
    U[4, 2, 5] = np.nan
    g.set_state(U)
    with pytest.raises(fr.FRError) as ei:
        g.residual()
    assert ei.value.name == "FR_ERR_NONFINITE"


def test_device_pointer_path():
    import torch

    fr = _fr()
    m = I.box_mesh(4, q=1)
    g = fr.FRMesh(m, 3, mu=1 / 1600)
    U = I.state_from_coords(g.sol_coords(), I.tgv_state)
    Ut = torch.from_numpy(U).cuda()
    g.set_state(Ut)
    Rt = torch.empty_like(Ut)
    g.residual(out=Rt)
    torch.cuda.synchronize()
    g.set_state(U)
    assert np.array_equal(Rt.cpu().numpy(), g.residual())


def test_degenerate_calls():
    """No elements is an argument error; zero RK steps leave the state bit for bit; the tuning
    calls reject arguments outside their ranges."""
    fr = _fr()
    m = I.box_mesh(3, q=1)
    empty = I.Mesh(elem_vert=m.elem_vert[:0].copy(), elem_nodes=m.elem_nodes[:0].copy(), q=1)
    with pytest.raises(fr.FRError) as ei:
        fr.FRMesh(empty, 2)
    assert ei.value.name == "FR_ERR_ARG"
    g = fr.FRMesh(m, 2, mu=1e-3)
    X = g.sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=1, amp=0.01)
    g.set_state(U)
    for scheme in ("lsrk45", "rk4", "ssprk104"):
        g.rk_step(1e-3, scheme, 0)
        assert np.array_equal(g.get_state(), U)
    with pytest.raises(fr.FRError) as ei:
        g.rk_step(1e-3, "lsrk45", -1)
    assert ei.value.name == "FR_ERR_ARG"
    with pytest.raises(fr.FRError) as ei:
        fr._check(fr.load().fr_autotune(g.h, 0, None))
    assert ei.value.name == "FR_ERR_ARG"
    with pytest.raises(fr.FRError):
        g.set_tiles(0, 3)
    with pytest.raises(fr.FRError):
        fr._check(fr.load().fr_set_fusion(g.h, -1))
    g.close()
