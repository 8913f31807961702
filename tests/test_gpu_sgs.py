"""GPU parity of the learned eddy-viscosity closure against the oracle, through the C ABI.

Tolerances and where they come from:
* features: FP64 on both sides, rounded to float32 once by the library; 3 float32 ulps plus
  1e-7 absolute (the logarithm of an energy near the 1e-12 floor amplifies FP64 round-off);
* residual with a given per-element nu_t: the FP64 floor rule of the plain residual
  (e_v <= max(1e-12, 2 f_v) against the long-double oracle);
* network forward: activations enter the bf16 products as hi + lo (relative error <= 2^-17)
  and products accumulate in float32 over K <= 128 terms (<= 128 * 2^-24 ~ 8e-6 of the sum of
  magnitudes); through two tanh layers and the softplus output this bounds |y_gpu - y| well
  below 1e-4 of max|y|, the gate used here;
* gradients: the same arithmetic plus float32 sums over the batch; each parameter block is
  gated at 5e-5 of its largest magnitude (five times the largest error measured, 9.5e-6 in W1:
  the hi + lo split's 2^-17 and the float32 sums) and the loss at 1e-5 relative;
* Adam: with the oracle's gradient the masters agree to 0.1 % of a step where that gradient is
  not negligible (elsewhere its sign is within the gradient's rounding and a step may differ);
  with the library's own gradient handed to the oracle's Adam, the float32 update agrees to
  2e-5 of the learning rate plus one float32 ulp per step, everywhere;
* bf16 weight copies: integer work, bit-exact against the oracle's rounding of the masters.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as M
from paper_2308_06605_amd import inputs as I

pytestmark = pytest.mark.gpu

MU = 1.0 / 1600.0


def _fr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_06605_amd import fr

    fr.load()
    return fr


def rel(a, b):
    return np.abs(a - b).max(axis=(0, 2)) / np.maximum(np.abs(b).max(axis=(0, 2)), 1e-300)


def _state(X, seed=4, amp=0.05):
    return I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=seed, amp=amp)


def _features_data(F, n, seed):
    rng = np.random.default_rng(seed)
    X = (rng.normal(size=(n, F)) * rng.uniform(0.5, 3, F) + rng.normal(size=F) * 4).astype(np.float32)
    mean = X.mean(axis=0).astype(np.float32)
    std = (X.std(axis=0) + 0.05).astype(np.float32)
    t = rng.uniform(0, 4, n).astype(np.float32)
    return X, mean, std, t


# ------------------------------------------------------------------------------ features
@pytest.mark.parametrize("p,n,curved", [(3, 5, True), (2, 4, False), (4, 3, True), (1, 4, True)])
def test_features_parity(p, n, curved):
    fr = _fr()
    m = I.box_mesh(n, q=min(p, 3) if curved else 1, curve_amp=0.05 if curved else 0.0, curve_mode="mixed")
    g = fr.FRMesh(m, p, mu=MU, flux="roe")
    X = g.sol_coords()
    U = _state(X)
    g.set_state(U)
    f = g.sgs_features().cpu().numpy()
    g.close()
    fo = oracle.Oracle(m, p, precision="ld").sgs_features(U)
    assert f.shape == fo.shape == (m.n_elem, (p + 1) ** 3 + 4)
    ref = fo.astype(np.float32)
    ulp = np.spacing(np.abs(ref)).astype(np.float64)
    err = np.abs(f.astype(np.float64) - fo)
    print(f"p={p} features max err {err.max():.3g}, max err/ulp {(err / (ulp + 1e-30)).max():.2f}", flush=True)
    assert np.all(err <= 3 * ulp + 1e-7), np.argwhere(err > 3 * ulp + 1e-7)[:5]


# ------------------------------------------------------------------------------ residual with nu_t
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_residual_fixed_eddy_viscosity(flux):
    fr = _fr()
    p = 3
    m = I.box_mesh(5, q=3, curve_amp=0.05, curve_mode="mixed")
    nu = np.random.default_rng(7).uniform(0, 0.01, m.n_elem)
    g = fr.FRMesh(m, p, mu=MU, flux=flux)
    X = g.sol_coords()
    U = _state(X)
    g.set_state(U)
    g.set_eddy_viscosity(nu, prandtl_t=0.9)
    R = g.residual()
    assert np.array_equal(g.eddy_viscosity(), nu)
    g.set_eddy_viscosity(None)
    R0 = g.residual()
    g.close()
    res = {}
    for prec in ("f64", "ld"):
        o = oracle.Oracle(m, p, mu=MU, flux=flux, precision=prec)
        o.set_eddy_viscosity(nu, 0.9)
        res[prec] = o.residual(U)
    e, f = rel(R, res["ld"]), rel(res["f64"], res["ld"])
    print(f"{flux} nu_t residual err {e} floor {f}", flush=True)
    assert np.all(e <= np.maximum(1e-12, 2 * f)), (e, f)
    # the closure changes the result, and switching it off restores the plain residual
    assert rel(R, R0).max() > 1e-6
    Rp = oracle.Oracle(m, p, mu=MU, flux=flux, precision="ld").residual(U)
    assert np.all(rel(R0, Rp) <= np.maximum(1e-12, 2 * rel(oracle.Oracle(m, p, mu=MU, flux=flux).residual(U), Rp)))


def test_eddy_viscosity_inviscid_mesh():
    """mu = 0 with a closure: the viscous path switches on for the eddy viscosity alone."""
    fr = _fr()
    p = 2
    m = I.box_mesh(4, q=2, curve_amp=0.05)
    nu = np.random.default_rng(1).uniform(0.001, 0.01, m.n_elem)
    g = fr.FRMesh(m, p, mu=0.0, flux="rusanov")
    U = _state(g.sol_coords())
    g.set_state(U)
    g.set_eddy_viscosity(nu)
    R = g.residual()
    g.close()
    res = {}
    for prec in ("f64", "ld"):
        o = oracle.Oracle(m, p, mu=0.0, flux="rusanov", precision=prec)
        o.set_eddy_viscosity(nu, 0.9)
        res[prec] = o.residual(U)
    e, f = rel(R, res["ld"]), rel(res["f64"], res["ld"])
    assert np.all(e <= np.maximum(1e-12, 2 * f)), (e, f)


# ------------------------------------------------------------------------------ network
@pytest.mark.parametrize("F,n", [(68, 1000), (13, 37), (128, 64), (31, 1)])
def test_mlp_forward_and_bf16_copies(F, n):
    import torch

    fr = _fr()
    X, mean, std, _ = _features_data(F, n, seed=F)
    theta = M.init_params(F, seed=3)
    net = fr.MLP(F, theta, mean, std)
    W1, W2, w3 = net.get_bf16()
    d = M.unpack(theta, F)
    assert np.array_equal(W1, (M.bf16_round(d["W1"]).view(np.uint32) >> 16).astype(np.uint16))
    assert np.array_equal(W2, (M.bf16_round(d["W2"]).view(np.uint32) >> 16).astype(np.uint16))
    assert np.array_equal(w3, (M.bf16_round(d["w3"]).view(np.uint32) >> 16).astype(np.uint16))
    Xd = torch.from_numpy(X).cuda()
    y = net.forward(Xd).cpu().numpy().astype(np.float64)
    yo = M.forward(M.effective(theta, F), X, mean, std)
    err = np.abs(y - yo).max() / np.abs(yo).max()
    print(f"F={F} n={n} forward rel err {err:.3g}", flush=True)
    assert err < 1e-4
    # a strided input (ldx > n_in) gives the same result
    Xw = torch.zeros((n, F + 7), dtype=torch.float32, device="cuda")
    Xw[:, :F] = Xd
    assert torch.equal(net.forward(Xw[:, :F]), net.forward(Xd))
    net.close()


def test_mlp_empty_batch_and_errors():
    import torch

    fr = _fr()
    F = 8
    theta = M.init_params(F, 0)
    net = fr.MLP(F, theta, np.zeros(F), np.ones(F))
    out = torch.full((1,), 7.0, device="cuda")
    net.forward(torch.zeros((0, F), device="cuda"), out=out)
    assert out.item() == 7.0
    with pytest.raises(fr.FRError):
        fr.MLP(F, theta, np.zeros(F), np.r_[np.ones(F - 1), 0.0])  # std must be > 0
    with pytest.raises(fr.FRError):
        fr.MLP(129, M.init_params(129, 0), np.zeros(129), np.ones(129))
    with pytest.raises(fr.FRError):
        net.train_step(torch.zeros((4, F), device="cuda"), torch.zeros(4, device="cuda"), lr=0.0)
    net.close()


@pytest.mark.parametrize("F,n", [(68, 700), (20, 33)])
def test_mlp_gradient_parity(F, n):
    import torch

    fr = _fr()
    X, mean, std, t = _features_data(F, n, seed=11 + F)
    theta = M.init_params(F, seed=5)
    net = fr.MLP(F, theta, mean, std)
    loss, g = net.loss_grad(torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda())
    Lo, go = M.loss_and_grad(theta, X, t, mean, std)
    assert abs(loss - Lo) <= 1e-5 * Lo, (loss, Lo)
    gd, god = M.unpack(g.astype(np.float64), F), M.unpack(go, F)
    for k in god:
        err = np.abs(gd[k] - god[k]).max() / np.abs(god[k]).max()
        print(f"F={F} grad {k} rel err {err:.3g}", flush=True)
        assert err < 5e-5, (k, err)
    # loss_grad does not update
    assert np.array_equal(net.get_params(), theta)
    net.close()


def test_mlp_adam_steps_match_oracle():
    import torch

    fr = _fr()
    F, n = 68, 512
    X, mean, std, t = _features_data(F, n, seed=2)
    theta = M.init_params(F, seed=9)
    net = fr.MLP(F, theta, mean, std)
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    opt = M.Adam(theta, lr=1e-3)
    loss_d = torch.zeros(1, device="cuda")
    for k in range(4):
        Lo, go = M.loss_and_grad(opt.theta, X, t, mean, std)
        net.train_step(Xd, td, 1e-3, loss_out=loss_d)
        opt.step(go)
        assert abs(loss_d.item() - Lo) <= 2e-5 * Lo, (k, loss_d.item(), Lo)
        th = net.get_params().astype(np.float64)
        # Adam's step is lr * m/(sqrt(v)+eps): insensitive to the gradient's last digits except
        # where the gradient is ~0; compare where the oracle's gradient is not negligible
        # (the first moment can cancel over steps, so the bound is 0.1 % of a step per step)
        lr = 1e-3
        big = np.abs(go) > 1e-4 * np.abs(go).max()
        diff = np.abs(th - opt.theta.astype(np.float64))
        assert np.all(diff[big] <= 1e-3 * lr * (k + 1) + 4 * np.spacing(np.abs(opt.theta[big]))), k
        assert np.all(diff <= 2 * lr * (k + 1) + 4 * np.spacing(np.abs(opt.theta)))
    # the bf16 copies follow the updated masters bit for bit
    W1, W2, w3 = net.get_bf16()
    d = M.unpack(net.get_params(), F)
    assert np.array_equal(W1, (M.bf16_round(d["W1"]).view(np.uint32) >> 16).astype(np.uint16))
    assert np.array_equal(W2, (M.bf16_round(d["W2"]).view(np.uint32) >> 16).astype(np.uint16))
    net.close()


def test_mlp_adam_update_from_its_own_gradient():
    """The Adam arithmetic alone: before each step the library's gradient at the current
    parameters (fr_mlp_loss_grad; the kernels have no atomics, so fr_mlp_train_step sums the same
    gradient) is handed to the oracle's Adam, whose float64 moments and update then differ from
    the library's float32 ones by rounding only: |m/(sqrt(v)+eps)| <= 3.2 for these betas and a
    float32 update is good to a few ulps of that, so per step at most 2e-5 of the learning rate,
    plus one float32 ulp of the parameter from the rounding of the masters."""
    import torch

    fr = _fr()
    F, n, lr = 68, 512, 1e-3
    X, mean, std, t = _features_data(F, n, seed=3)
    theta = M.init_params(F, seed=4)
    net = fr.MLP(F, theta, mean, std)
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    opt = M.Adam(theta, lr=lr)
    for k in range(6):
        _, g = net.loss_grad(Xd, td)
        net.train_step(Xd, td, lr)
        opt.step(g.astype(np.float64))
        th = net.get_params().astype(np.float64)
        diff = np.abs(th - opt.theta.astype(np.float64))
        bound = (k + 1) * (2e-5 * lr + np.spacing(np.abs(opt.theta)).astype(np.float64))
        print(f"Adam step {k}: max |diff| / bound {(diff / bound).max():.3g}", flush=True)
        assert np.all(diff <= bound), (k, (diff / bound).max())
    net.close()


def test_mlp_training_reduces_loss():
    import torch

    fr = _fr()
    F, n = 12, 2048
    rng = np.random.default_rng(0)
    X = rng.normal(size=(n, F)).astype(np.float32)
    t = (np.log1p(np.exp(X[:, 0] - 0.5 * X[:, 1] ** 2 + 0.3 * X[:, 2] * X[:, 3]))).astype(np.float32)
    net = fr.MLP(F, M.init_params(F, 1), np.zeros(F), np.ones(F))
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    L0, _ = net.loss_grad(Xd, td)
    for _ in range(400):
        net.train_step(Xd, td, 3e-3)
    L1, _ = net.loss_grad(Xd, td)
    print(f"loss {L0:.4g} -> {L1:.4g}", flush=True)
    assert L1 < 0.1 * L0
    net.close()


# ------------------------------------------------------------------------------ model attached
def _model_for(F, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    theta = M.init_params(F, seed)
    d = M.unpack(theta, F)
    d["b3"][:] = -1.0
    d["w3"] *= scale
    return M.pack(d).astype(np.float32)


def test_residual_with_model_matches_oracle():
    fr = _fr()
    p = 3
    m = I.box_mesh(4, q=3, curve_amp=0.05, curve_mode="mixed")
    g = fr.FRMesh(m, p, mu=MU, flux="roe")
    X = g.sol_coords()
    U = _state(X)
    g.set_state(U)
    F = g.n_features
    feats = g.sgs_features().cpu().numpy()
    mean, std = feats.mean(axis=0), feats.std(axis=0) + 0.1
    theta = _model_for(F, 3)
    net = fr.MLP(F, theta, mean, std)
    nu_scale = 0.004
    g.set_sgs_model(net, nu_scale=nu_scale, prandtl_t=0.9)
    R = g.residual()
    nu = g.eddy_viscosity()
    g.close()
    net.close()
    # nu_t from the oracle's features (rounded to float32 as the library stores them) and network
    fo = oracle.Oracle(m, p, precision="ld").sgs_features(U).astype(np.float32)
    nu_o = nu_scale * M.forward(M.effective(theta, F), fo, mean.astype(np.float32), std.astype(np.float32))
    enu = np.abs(nu - nu_o).max() / np.abs(nu_o).max()
    print(f"model nu_t rel err {enu:.3g}, nu range {nu.min():.3g}..{nu.max():.3g}", flush=True)
    assert enu < 1e-4
    # the residual for the library's nu_t meets the FP64 floor rule
    res = {}
    for prec in ("f64", "ld"):
        o = oracle.Oracle(m, p, mu=MU, flux="roe", precision=prec)
        o.set_eddy_viscosity(nu, 0.9)
        res[prec] = o.residual(U)
    e, f = rel(R, res["ld"]), rel(res["f64"], res["ld"])
    assert np.all(e <= np.maximum(1e-12, 2 * f)), (e, f)


def test_rk_step_with_model_evaluates_each_stage():
    """One RK4 step with the model attached against an oracle RK4 whose every stage computes
    the features and nu_t of its own stage state; compared relative to the step's increment."""
    fr = _fr()
    p, dt = 3, 2e-3
    m = I.box_mesh(4, q=1)
    g = fr.FRMesh(m, p, mu=MU, flux="rusanov")
    X = g.sol_coords()
    U0 = _state(X, amp=0.1)
    g.set_state(U0)
    F = g.n_features
    feats = g.sgs_features().cpu().numpy()
    mean, std = feats.mean(axis=0), feats.std(axis=0) + 0.1
    theta = _model_for(F, 8, scale=3.0)
    net = fr.MLP(F, theta, mean, std)
    nu_scale = 0.01
    g.set_sgs_model(net, nu_scale=nu_scale)
    g.rk_step(dt, "rk4", 1)
    U1 = g.get_state()
    g.close()
    net.close()
    o = oracle.Oracle(m, p, mu=MU, flux="rusanov")
    eff = M.effective(theta, F)

    def rhs(U):
        f = o.sgs_features(U).astype(np.float32)
        o.set_eddy_viscosity(nu_scale * M.forward(eff, f, mean.astype(np.float32), std.astype(np.float32)), 0.9)
        return o.residual(U)

    k1 = rhs(U0)
    k2 = rhs(U0 + 0.5 * dt * k1)
    k3 = rhs(U0 + 0.5 * dt * k2)
    k4 = rhs(U0 + dt * k3)
    Uo = U0 + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    # frozen nu_t (first stage only) for contrast: the per-stage evaluation must be closer
    o.set_eddy_viscosity(None)
    nu0 = nu_scale * M.forward(eff, o.sgs_features(U0).astype(np.float32), mean.astype(np.float32),
                               std.astype(np.float32))
    o.set_eddy_viscosity(nu0, 0.9)
    Uf = o.rk_step(U0, dt, "rk4", 1)
    inc = np.abs(Uo - U0).max(axis=(0, 2))
    e = np.abs(U1 - Uo).max(axis=(0, 2)) / inc
    e_frozen = np.abs(Uf - Uo).max(axis=(0, 2)) / inc
    print(f"rk4 with model: err/increment {e}, frozen-nu difference {e_frozen}", flush=True)
    assert np.all(e < 1e-5), e
    assert e_frozen.max() > 10 * e.max()


def test_closure_error_paths():
    fr = _fr()
    m = I.box_mesh(3, q=1)
    g32 = fr.FRMesh(m, 3, mu=MU, prec="fp32", ref_rho=1.0, ref_p=71.4)
    with pytest.raises(fr.FRError) as ei:
        g32.set_eddy_viscosity(np.zeros(m.n_elem))
    assert ei.value.name == "FR_ERR_UNSUPPORTED"
    g32.close()
    g = fr.FRMesh(m, 3, mu=MU)
    with pytest.raises(fr.FRError):
        g.set_eddy_viscosity(np.full(m.n_elem, -1.0))
    with pytest.raises(fr.FRError):
        g.set_eddy_viscosity(np.zeros(m.n_elem), prandtl_t=0.0)
    net = fr.MLP(10, M.init_params(10, 0), np.zeros(10), np.ones(10))
    with pytest.raises(fr.FRError):
        g.set_sgs_model(net, 1.0)  # wrong input size
    with pytest.raises(fr.FRError):
        g.eddy_viscosity()  # nothing set yet
    net.close()
    g.close()
