"""Pins for the oracle's learned-closure pieces: the per-element features, the residual with a
per-element eddy viscosity, and the network (forward, gradient, Adam).

What fixes each one independently of the oracle's own code:
* features: a single orthonormal Legendre mode has a closed-form energy; Parseval's identity
  under the exact Gauss quadrature; a linear velocity field on trilinear elements has an exactly
  known gradient, so every invariant is known in closed form; adding a constant velocity changes
  nothing; the invariants do not depend on element labels or reference-frame rotations;
* eddy viscosity: zero reproduces the plain residual bit for bit; a uniform nu_t on a
  constant-density state is the plain residual with mu + nu_t (and the matching Prandtl number);
  discrete conservation and relabel/rotation invariance hold for a random per-element nu_t;
* network: bf16 rounding equals torch's float32 -> bfloat16 conversion; the forward pass equals
  a torch.nn stack; gradients equal torch autograd and central finite differences; Adam equals
  torch.optim.Adam.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as M
from paper_2308_06605_amd import inputs as I

MU = 0.01


def gl(p):
    return np.polynomial.legendre.leggauss(p + 1)


def onl(a, x):
    """orthonormal Legendre polynomial on [-1, 1]"""
    c = np.zeros(a + 1)
    c[a] = 1.0
    return np.sqrt((2 * a + 1) / 2) * np.polynomial.legendre.legval(x, c)


def ref_points(p):
    x = gl(p)[0]
    k, j, i = np.meshgrid(x, x, x, indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


def state_with_velocity(o, u):
    """rho = 1, p = 50, velocity u [E][3][Ns]"""
    E, Ns = u.shape[0], u.shape[2]
    U = np.zeros((E, 5, Ns))
    U[:, 0] = 1.0
    U[:, 1:4] = u
    U[:, 4] = 50.0 / 0.4 + 0.5 * (u ** 2).sum(axis=1)
    return U


# ---------------------------------------------------------------------- features
@pytest.mark.parametrize("p", [2, 3])
def test_single_mode_energy(p):
    m = I.box_mesh(3, q=1)
    o = oracle.Oracle(m, p)
    n = p + 1
    xi, eta, zeta = ref_points(p)
    modes = [(1, 0, 0), (0, 2, 1), (p, p, p), (1, 1, 0)]
    u = np.zeros((m.n_elem, 3, n ** 3))
    picks = {}
    for e in range(m.n_elem):
        a, b, c = modes[e % len(modes)]
        amp = 0.3 + 0.1 * e
        comp = e % 3
        u[e, comp] = amp * onl(a, xi) * onl(b, eta) * onl(c, zeta)
        picks[e] = ((a, b, c), amp)
    f = o.sgs_features(state_with_velocity(o, u))
    assert f.shape == (m.n_elem, n ** 3 + 4)
    for e, ((a, b, c), amp) in picks.items():
        k = a + n * (b + n * c) - 1  # the constant mode is dropped
        e_exp = amp ** 2 / 16
        assert abs(f[e, k] - np.log(e_exp + 1e-12)) < 1e-12
        others = np.delete(f[e, : n ** 3 - 1], k)
        assert np.all(others < np.log(1e-12) + 1e-6)  # zero energy -> ln(eps)


def test_parseval():
    p = 3
    m = I.box_mesh(3, q=3, curve_amp=0.05)
    o = oracle.Oracle(m, p)
    X = o.sol_coords()
    rng = np.random.default_rng(0)
    u = rng.normal(size=(m.n_elem, 3, 64))
    f = o.sgs_features(state_with_velocity(o, u))
    e = np.exp(f[:, :63]) - 1e-12
    w = gl(p)[1]
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    mean = np.einsum("ejs,s->ej", u, W) / 8
    total = np.einsum("ejs,s->e", 0.5 * u ** 2, W) / 8
    assert np.allclose(e.sum(axis=1), total - 0.5 * (mean ** 2).sum(axis=1), rtol=1e-12, atol=1e-14)
    assert X.shape[0] == m.n_elem


def _linear_field_case(seed):
    p = 3
    m = I.box_mesh(3, q=1, curve_amp=0.08, curve_mode="mixed")  # trilinear (non-affine) elements
    o = oracle.Oracle(m, p)
    X = o.sol_coords()
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(3, 3))  # A[i][j] = d u_j / d x_i
    u0 = rng.normal(size=3)
    u = np.einsum("eis,ij->ejs", X, A) + u0[None, :, None]
    return o, A, u


def test_linear_field_invariants_exact():
    o, A, u = _linear_field_case(1)
    f = o.sgs_features(state_with_velocity(o, u))
    S, W = (A + A.T) / 2, (A - A.T) / 2
    s2, w2 = 2 * (S * S).sum(), 2 * (W * W).sum()
    r = -np.trace(A @ A @ A) / 3
    th = np.trace(A)
    exp = [np.log(s2 + 1e-12) / 2, np.log(w2 + 1e-12) / 2, r / (s2 + 1e-12) ** 1.5,
           th / np.sqrt(s2 + 1e-12), th * th / (s2 + 1e-12)]
    assert np.allclose(f[:, 63:], np.array(exp)[None, :], rtol=1e-10, atol=1e-11)


def test_galilean_invariance():
    o, A, u = _linear_field_case(2)
    rng = np.random.default_rng(3)
    u = u + 0.1 * rng.normal(size=u.shape)
    f1 = o.sgs_features(state_with_velocity(o, u))
    f2 = o.sgs_features(state_with_velocity(o, u + np.array([0.7, -0.2, 0.4])[None, :, None]))
    # modal energies of non-constant modes and the gradient do not see a constant velocity;
    # a tiny energy's logarithm amplifies the round-off of the shifted field
    e1, e2 = np.exp(f1[:, :63]), np.exp(f2[:, :63])
    assert np.allclose(e1, e2, rtol=1e-9, atol=1e-15)
    assert np.allclose(f1[:, 63:], f2[:, 63:], rtol=1e-10, atol=1e-12)


def test_invariants_relabel_rotate():
    p = 3
    m = I.box_mesh(3, q=3, curve_amp=0.05, curve_mode="mixed")
    ms, info = I.scramble_mesh(m, seed=4)
    o = oracle.Oracle(m, p, precision="ld")
    X = o.sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=2, amp=0.05)
    f = o.sgs_features(U)
    o2 = oracle.Oracle(ms, p, precision="ld")
    f2 = o2.sgs_features(I.scramble_field(U, info, p))
    order = info[0]
    assert np.allclose(f2[:, 63:], f[order, 63:], rtol=1e-12, atol=1e-13)
    # the modal energies are permuted among modes of the same (sorted) degree triple
    n = p + 1
    deg = [tuple(sorted((a, b, c))) for c in range(n) for b in range(n) for a in range(n)][1:]
    for key in set(deg):
        idx = [i for i, d in enumerate(deg) if d == key]
        assert np.allclose(np.sort(np.exp(f2[:, idx]), axis=1), np.sort(np.exp(f[order][:, idx]), axis=1),
                           rtol=1e-10, atol=1e-16)


# ---------------------------------------------------------------------- eddy viscosity
def test_zero_eddy_viscosity_is_plain():
    m = I.box_mesh(3, q=3, curve_amp=0.05)
    o = oracle.Oracle(m, 3, mu=MU, flux="roe")
    U = I.state_from_coords(o.sol_coords(), I.tgv_state)
    R0 = o.residual(U)
    o.set_eddy_viscosity(np.zeros(m.n_elem))
    assert np.array_equal(o.residual(U), R0)


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_uniform_eddy_viscosity_constant_density(flux):
    p, nu, prt, pr = 3, 0.02, 0.9, 0.72
    m = I.box_mesh(3, q=3, curve_amp=0.05, curve_mode="mixed")
    o = oracle.Oracle(m, p, mu=MU, flux=flux, prandtl=pr, precision="ld")
    X = o.sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=7, amp=0.02)
    rho = U[:, 0:1].copy()
    U[:, 1:4] /= rho
    U[:, 4] = U[:, 4] / rho[:, 0]  # rescale to rho = 1 keeping velocity and temperature
    U[:, 0] = 1.0
    o.set_eddy_viscosity(np.full(m.n_elem, nu), prt)
    R = o.residual(U)
    mu2 = MU + nu
    pr2 = mu2 / (MU / pr + nu / prt)
    R2 = oracle.Oracle(m, p, mu=mu2, flux=flux, prandtl=pr2, precision="ld").residual(U)
    err = np.abs(R - R2).max(axis=(0, 2)) / np.abs(R2).max(axis=(0, 2)).clip(1e-300)
    assert np.all(err[1:] < 1e-13), err
    assert np.abs(R[:, 0] - R2[:, 0]).max() < 1e-13 * np.abs(R2).max()


def test_eddy_viscosity_conservation():
    p = 3
    m = I.box_mesh(4, q=3, curve_amp=0.05, curve_mode="mixed")
    o = oracle.Oracle(m, p, mu=MU, flux="roe")
    X = o.sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=3, amp=0.01)
    o.set_eddy_viscosity(np.random.default_rng(1).uniform(0, 0.05, m.n_elem))
    R = o.residual(U)
    _, dJ, _, _ = o.geometry()
    w = gl(p)[1]
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    tot = np.einsum("evs,es,s->v", R, dJ, W)
    mag = np.einsum("evs,es,s->v", np.abs(R), dJ, W)
    assert np.all(np.abs(tot) / mag < 1e-12), tot / mag


def test_eddy_viscosity_relabel_rotate():
    p = 3
    m = I.box_mesh(3, q=3, curve_amp=0.05, curve_mode="mixed")
    ms, info = I.scramble_mesh(m, seed=8)
    nu = np.random.default_rng(2).uniform(0, 0.05, m.n_elem)
    o = oracle.Oracle(m, p, mu=MU, flux="roe", precision="ld")
    X = o.sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=5, amp=0.02)
    o.set_eddy_viscosity(nu)
    R = o.residual(U)
    o2 = oracle.Oracle(ms, p, mu=MU, flux="roe", precision="ld")
    o2.set_eddy_viscosity(nu[info[0]])
    R2 = o2.residual(I.scramble_field(U, info, p))
    Rs = I.scramble_field(R, info, p)
    err = np.abs(R2 - Rs).max(axis=(0, 2)) / np.abs(Rs).max(axis=(0, 2))
    assert np.all(err < 5e-13), err


def test_eddy_viscosity_dissipates_kinetic_energy():
    """A positive eddy viscosity removes kinetic energy: d/dt of the quadrature kinetic energy
    is lower with nu_t > 0 than without, for a smooth periodic flow."""
    p = 3
    m = I.box_mesh(4, q=1)
    o = oracle.Oracle(m, p, mu=MU, flux="roe")
    U = I.state_from_coords(o.sol_coords(), I.tgv_state)
    _, dJ, _, _ = o.geometry()
    w = gl(p)[1]
    W = np.einsum("k,j,i->kji", w, w, w).ravel()[None, :] * dJ

    def dek(R):
        rho, mom = U[:, 0], U[:, 1:4]
        q2 = (mom ** 2).sum(axis=1) / rho ** 2
        return (W * ((mom * R[:, 1:4]).sum(axis=1) / rho - 0.5 * q2 * R[:, 0])).sum()

    d0 = dek(o.residual(U))
    o.set_eddy_viscosity(np.full(m.n_elem, 0.05))
    d1 = dek(o.residual(U))
    assert d1 < d0 < 0


def test_negative_eddy_viscosity_rejected():
    m = I.box_mesh(3, q=1)
    o = oracle.Oracle(m, 2, mu=MU)
    with pytest.raises(RuntimeError):
        o.set_eddy_viscosity(np.full(m.n_elem, -1.0))


# ---------------------------------------------------------------------- network
def test_bf16_round_matches_torch():
    import torch

    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000).astype(np.float32) * 10.0 ** rng.integers(-8, 8, 4000),
                        np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0, -0.0,
                                  1 + 2 ** -8 + 2 ** -20, 3.0e38], dtype=np.float32)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(M.bf16_round(x).view(np.uint32), ref.view(np.uint32))


def _net(F=12, N=37, seed=0):
    rng = np.random.default_rng(seed)
    theta = M.init_params(F, seed)
    X = rng.normal(size=(N, F)).astype(np.float32) * 2 + 1
    mean = X.mean(axis=0).astype(np.float32)
    std = (X.std(axis=0) + 0.1).astype(np.float32)
    t = rng.uniform(0, 3, N).astype(np.float32)
    return theta, X, t, mean, std


def _torch_net(eff, F):
    import torch

    net = torch.nn.Sequential(torch.nn.Linear(F, M.H), torch.nn.Tanh(), torch.nn.Linear(M.H, M.H),
                              torch.nn.Tanh(), torch.nn.Linear(M.H, 1), torch.nn.Softplus()).double()
    with torch.no_grad():
        net[0].weight.copy_(torch.from_numpy(eff["W1"]))
        net[0].bias.copy_(torch.from_numpy(eff["b1"]))
        net[2].weight.copy_(torch.from_numpy(eff["W2"]))
        net[2].bias.copy_(torch.from_numpy(eff["b2"]))
        net[4].weight.copy_(torch.from_numpy(eff["w3"][None, :]))
        net[4].bias.copy_(torch.from_numpy(eff["b3"]))
    return net


def test_forward_matches_torch():
    import torch

    theta, X, t, mean, std = _net()
    F = X.shape[1]
    eff = M.effective(theta, F)
    y = M.forward(eff, X, mean, std)
    net = _torch_net(eff, F)
    xh = (X.astype(np.float64) - mean) / std.astype(np.float64)
    y_t = net(torch.from_numpy(xh)).detach().numpy()[:, 0]
    assert np.allclose(y, y_t, rtol=1e-14, atol=1e-15)
    # the weights it used are bf16 values
    assert np.array_equal(M.bf16_round(eff["W1"].astype(np.float32)), eff["W1"].astype(np.float32))


def test_gradient_matches_torch_autograd():
    import torch

    theta, X, t, mean, std = _net(seed=3)
    F = X.shape[1]
    L, g = M.loss_and_grad(theta, X, t, mean, std)
    eff = M.effective(theta, F)
    net = _torch_net(eff, F)
    xh = torch.from_numpy((X.astype(np.float64) - mean) / std.astype(np.float64))
    loss = ((net(xh)[:, 0] - torch.from_numpy(t.astype(np.float64))) ** 2).mean()
    loss.backward()
    gt = M.pack({"W1": net[0].weight.grad.numpy(), "b1": net[0].bias.grad.numpy(),
                 "W2": net[2].weight.grad.numpy(), "b2": net[2].bias.grad.numpy(),
                 "w3": net[4].weight.grad.numpy()[0], "b3": net[4].bias.grad.numpy()})
    assert abs(L - loss.item()) < 1e-14 * abs(L)
    assert np.allclose(g, gt, rtol=1e-12, atol=1e-15 * np.abs(gt).max())


def test_gradient_finite_differences():
    theta, X, t, mean, std = _net(F=6, N=9, seed=5)
    F = X.shape[1]
    L, g = M.loss_and_grad(theta, X, t, mean, std)
    eff = M.effective(theta, F)
    flat = M.pack(eff)
    rng = np.random.default_rng(1)
    for i in rng.choice(flat.size, 40, replace=False):
        h = 1e-6
        vals = []
        for s in (1, -1):
            f2 = flat.copy()
            f2[i] += s * h
            e2 = M.unpack(f2, F)
            vals.append(np.mean((M.forward(e2, X, mean, std) - t) ** 2))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 * max(1.0, abs(g).max()), (i, fd, g[i])


def test_adam_matches_torch():
    import torch

    theta, X, t, mean, std = _net(seed=9)
    opt = M.Adam(theta, lr=1e-2)
    p = torch.nn.Parameter(torch.from_numpy(theta.astype(np.float64)))
    topt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    rng = np.random.default_rng(0)
    for k in range(5):
        g = rng.normal(size=theta.size) * 10.0 ** rng.integers(-6, 1, theta.size)
        opt.step(g)
        topt.zero_grad()
        p.grad = torch.from_numpy(g)
        topt.step()
        with torch.no_grad():
            p.copy_(p.float().double())  # masters are float32
        assert np.array_equal(opt.theta, p.detach().numpy().astype(np.float32)), k
    # the first step moves every parameter with a nonzero gradient by lr (bias-corrected moments)
    opt2 = M.Adam(theta, lr=1e-3)
    g = np.where(np.arange(theta.size) % 3 == 0, 0.0, rng.normal(size=theta.size))
    d = opt2.step(g).astype(np.float64) - theta
    nz = g != 0
    assert np.allclose(np.abs(d[nz]), 1e-3, rtol=1e-3)
    assert np.all(d[~nz] == 0)
