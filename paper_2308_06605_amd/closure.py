"""Learned eddy-viscosity closure: training data from the solver's own filtered high-order runs,
training with the library's network kernels, and the a-posteriori comparison with implicit LES.

The paper's solver supports LES sub-grid scale models (section "ZFR Framework") without
specifying one; this module builds a learned one on top of the library's closure entry points
(fr_sgs_features, fr_set_eddy_viscosity, fr_set_sgs_model, fr_mlp_*). Every flow computation
runs in libfr's kernels; numpy only moves data and applies the fine-to-coarse filter.

Setting (all on the periodic box [0, 2 pi)^3, Mach 0.1, Re = 5000, Roe + BR2, LSRK45):
  fine   32^3 elements, p = 7 (256 points per direction)
  coarse 16^3 elements, p = 3 (64 points per direction): each coarse element holds 2^3 fine ones
Filter P: the element-local L2 projection of the fine solution onto the coarse element's
degree-3 polynomials (exact Gauss quadrature on the fine points).
Target (training): the least-squares eddy viscosity of the filtered sub-grid stress,
tau_ij = P(u_i u_j) - P(u_i) P(u_j) ~ -2 nu_t S_ij^d with S the strain rate of P(u):
nu_t(e) = max(0, -<tau^d : S^d>_e / (2 <S^d : S^d>_e)) over the coarse element's points.
Diagnostic (stored, not trained on): the closure term the coarse discretisation misses,
C = P(R_fine(U_f)) - R_coarse(P U_f), projected on the residual response V = dR_coarse/d nu_t
to a uniform eddy viscosity, nu_c(e) = max(0, <C_m . V_m>_e / <V_m . V_m>_e). On these runs it
is zero almost everywhere: the coarse scheme's numerical dissipation acting on the projected
(element-wise discontinuous) field already exceeds the sub-grid energy transfer.
Features: fr_sgs_features of the coarse state P U_f. Network output y = nu_t / nu_scale with
nu_scale = mu (unit density).

Command line (GPU):
  python -m paper_2308_06605_amd.closure gen   --ic spectrum:SEED:K0:KMAX --t-end 1.5 --every 0.25 --out D.npz
  python -m paper_2308_06605_amd.closure gen   --ic tgv --t-end 6 --every 0.25 --out ref.npz
  python -m paper_2308_06605_amd.closure train --data D1.npz D2.npz ... --val Dv.npz --out model.npz
  python -m paper_2308_06605_amd.closure eval  --model model.npz --ref ref.npz
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs as I

GAMMA = 1.4
MACH = 0.1
RE = 5000.0
MU = 1.0 / RE
FLUX = "roe"
FINE = (32, 7)
COARSE = (16, 3)
RATIO = FINE[0] // COARSE[0]
DT_FINE = 2.5e-4
DT_COARSE = 1e-3
NU_SCALE = MU
PRANDTL_T = 0.9
NU_PROBE = 1e-3


def log(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------------------------------
# filter
# ------------------------------------------------------------------------------------------
def _onl(a, x):
    c = np.zeros(a + 1)
    c[a] = 1.0
    return np.sqrt((2 * a + 1) / 2.0) * np.polynomial.legendre.legval(x, c)


def restriction_1d(pc: int, pf: int, ratio: int) -> np.ndarray:
    """[pc+1][ratio*(pf+1)]: fine nodal values on `ratio` consecutive fine elements -> nodal
    values at the coarse Gauss points of their L2 projection onto degree pc."""
    xf, wf = np.polynomial.legendre.leggauss(pf + 1)
    xc = np.polynomial.legendre.leggauss(pc + 1)[0]
    xi = np.concatenate([-1.0 + (2 * r + xf + 1.0) / ratio for r in range(ratio)])
    w = np.tile(wf, ratio) / ratio
    Vc = np.stack([_onl(a, xc) for a in range(pc + 1)], axis=1)       # [coarse pt][mode]
    Vf = np.stack([_onl(a, xi) for a in range(pc + 1)], axis=0) * w   # [mode][fine pt]
    return Vc @ Vf


def restrict(Uf: np.ndarray, shape_f, pf: int, pc: int, ratio: int) -> np.ndarray:
    """Filter a state [Ef][C][(pf+1)^3] on an uncurved box of shape_f elements to the coarse box
    with ratio^3 fine elements per coarse element: [Ec][C][(pc+1)^3]."""
    nx, ny, nz = shape_f
    nf, nc = pf + 1, pc + 1
    C = Uf.shape[1]
    Rm = restriction_1d(pc, pf, ratio).reshape(nc, ratio, nf)
    T = Uf.reshape(nz // ratio, ratio, ny // ratio, ratio, nx // ratio, ratio, C, nf, nf, nf)
    T = np.tensordot(T, Rm, axes=([5, 9], [1, 2]))   # cz rz cy ry cx C k j a
    T = np.tensordot(T, Rm, axes=([3, 7], [1, 2]))   # cz rz cy cx C k a b
    T = np.tensordot(T, Rm, axes=([1, 5], [1, 2]))   # cz cy cx C a b c
    T = np.transpose(T, (0, 1, 2, 3, 6, 5, 4))
    return np.ascontiguousarray(T.reshape(-1, C, nc ** 3))


def quad_weights(p: int) -> np.ndarray:
    w = np.polynomial.legendre.leggauss(p + 1)[1]
    return np.einsum("k,j,i->kji", w, w, w).ravel()


def kinetic_energy(U: np.ndarray, p: int) -> float:
    """Volume-averaged rho |u|^2 / 2 of a state on an uncurved mesh (Gauss quadrature)."""
    W = quad_weights(p)
    e = 0.5 * (U[:, 1:4] ** 2).sum(axis=1) / U[:, 0]
    return float((e * W).sum() / (W.sum() * U.shape[0]))


# ------------------------------------------------------------------------------------------
# meshes and initial conditions
# ------------------------------------------------------------------------------------------
def _fr():
    from . import fr

    fr.load()
    return fr


def meshes():
    return I.box_mesh(FINE[0], q=1), I.box_mesh(COARSE[0], q=1)


def make_state(ic: str, mesh, g) -> np.ndarray:
    """ic = 'tgv' or 'spectrum:SEED:K0[:KMAX]'."""
    if ic == "tgv":
        return I.state_from_coords(g.sol_coords(), I.tgv_state, mach=MACH)
    parts = ic.split(":")
    assert parts[0] == "spectrum" and len(parts) in (3, 4)
    kmax = int(parts[3]) if len(parts) == 4 else 8
    return I.random_spectrum_state(mesh, g.p, seed=int(parts[1]), k0=float(parts[2]), kmax=kmax, mach=MACH)


# ------------------------------------------------------------------------------------------
# gen: training pairs (and the filtered reference) from a fine run
# ------------------------------------------------------------------------------------------
def deriv_1d(p: int) -> np.ndarray:
    """D[a][b] = l_b'(x_a) on the Gauss points of degree p."""
    x = np.polynomial.legendre.leggauss(p + 1)[0]
    n = p + 1
    D = np.zeros((n, n))
    for b in range(n):
        c = np.zeros(n)
        c[b] = 1.0
        # Lagrange basis l_b as a polynomial through the nodes
        lb = np.polynomial.polynomial.Polynomial.fit(x, c, p, domain=[-1, 1], window=[-1, 1])
        D[:, b] = lb.deriv()(x)
    return D


def stress_target(Uf: np.ndarray, shape_f, h_coarse: float):
    """Least-squares eddy viscosity of the filtered sub-grid stress per coarse element."""
    pf, pc = FINE[1], COARSE[1]
    n = pc + 1
    u = Uf[:, 1:4] / Uf[:, 0:1]
    ub = restrict(u, shape_f, pf, pc, RATIO)                        # [Ec][3][Ns]
    pairs = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    uu = np.stack([u[:, i] * u[:, j] for i, j in pairs], axis=1)
    uub = restrict(uu, shape_f, pf, pc, RATIO)
    del uu
    tau = np.zeros((ub.shape[0], 3, 3, ub.shape[2]))
    for k, (i, j) in enumerate(pairs):
        tau[:, i, j] = tau[:, j, i] = uub[:, k] - ub[:, i] * ub[:, j]
    D = deriv_1d(pc) * (2.0 / h_coarse)
    g = ub.reshape(-1, 3, n, n, n)                                  # e, comp, k(z), j(y), i(x)
    grad = np.stack([np.einsum("ai,eqkji->eqkja", D, g),          # d/dx
                     np.einsum("bj,eqkji->eqkbi", D, g),          # d/dy
                     np.einsum("ck,eqkji->eqcji", D, g)], axis=1)  # d/dz: [e][d][comp][z][y][x]
    A = grad.reshape(ub.shape[0], 3, 3, -1)                         # A[e][i][j] = d u_j / d x_i
    S = 0.5 * (A + np.transpose(A, (0, 2, 1, 3)))
    trS = (S[:, 0, 0] + S[:, 1, 1] + S[:, 2, 2]) / 3
    trT = (tau[:, 0, 0] + tau[:, 1, 1] + tau[:, 2, 2]) / 3
    for i in range(3):
        S[:, i, i] -= trS
        tau[:, i, i] -= trT
    W = quad_weights(pc)
    num = -np.einsum("eijs,eijs,s->e", tau, S, W)
    den = 2.0 * np.einsum("eijs,eijs,s->e", S, S, W)
    return np.maximum(0.0, num / np.maximum(den, 1e-300))


def targets_and_features(gc, Ub: np.ndarray, Rb: np.ndarray):
    """Per coarse element closure-term coefficient nu_c (diagnostic) and the library's features
    of the filtered state."""
    gc.set_eddy_viscosity(None)
    gc.set_state(Ub)
    R0 = gc.residual()
    gc.set_eddy_viscosity(np.full(gc.E, NU_PROBE), PRANDTL_T)
    R1 = gc.residual()
    gc.set_eddy_viscosity(None)
    Cm = (Rb - R0)[:, 1:4]
    Vm = ((R1 - R0) / NU_PROBE)[:, 1:4]
    W = quad_weights(COARSE[1])
    num = np.einsum("eis,eis,s->e", Cm, Vm, W)
    den = np.einsum("eis,eis,s->e", Vm, Vm, W)
    nut = np.maximum(0.0, num / np.maximum(den, 1e-300))
    feats = gc.sgs_features().cpu().numpy()
    return nut, feats, R0


def configure(fine=None, coarse=None):
    """Override the fine and coarse (elements per direction, degree) pairs (e.g. for a quick
    end-to-end check at small sizes)."""
    global FINE, COARSE, RATIO
    if fine:
        FINE = tuple(int(v) for v in fine)
    if coarse:
        COARSE = tuple(int(v) for v in coarse)
    assert FINE[0] % COARSE[0] == 0
    RATIO = FINE[0] // COARSE[0]


def gen(ic: str, t_end: float, every: float, out: str, keep_state_at=None, reference=False):
    fr = _fr()
    mf, mc = meshes()
    gf = fr.FRMesh(mf, FINE[1], mu=MU, flux=FLUX, check_finite=True)
    gc = fr.FRMesh(mc, COARSE[1], mu=MU, flux=FLUX)
    U0 = make_state(ic, mf, gf)
    gf.set_state(U0)
    steps = int(round(every / DT_FINE))
    nsnap = int(round(t_end / every))
    rec = {k: [] for k in ("t", "nut", "feats", "ek_filtered", "ek_fine", "dek_fine", "dek_coarse_filtered")}
    states = {}
    t0 = time.time()
    for s in range(nsnap + 1):
        if s > 0:
            gf.rk_step(DT_FINE, "lsrk45", steps)
        t = s * steps * DT_FINE
        Uf = gf.get_state()
        if not np.isfinite(Uf).all():
            raise FloatingPointError(f"non-finite fine state at t={t}")
        ek_f, dek_f = gf.kinetic_energy()
        Ub = restrict(Uf, mf.shape, FINE[1], COARSE[1], RATIO)
        if reference:
            # the filtered reference only: no targets
            nut, feats, dek_c = np.zeros(gc.E), np.zeros((gc.E, gc.n_features), np.float32), 0.0
        else:
            Rf = gf.residual()
            Rb = restrict(Rf, mf.shape, FINE[1], COARSE[1], RATIO)
            del Rf
            nuc, feats, R0 = targets_and_features(gc, Ub, Rb)
            nut = stress_target(Uf, mf.shape, (mc.hi[0] - mc.lo[0]) / COARSE[0])
            rec.setdefault("nu_closure", []).append(nuc)
            W = quad_weights(COARSE[1])
            rho, mom = Ub[:, 0], Ub[:, 1:4]
            q2 = (mom ** 2).sum(axis=1) / rho ** 2
            dek_c = float((W * ((mom * R0[:, 1:4]).sum(axis=1) / rho - 0.5 * q2 * R0[:, 0])).sum()
                          / (W.sum() * Ub.shape[0]))
        for k, v in (("t", t), ("nut", nut), ("feats", feats), ("ek_filtered", kinetic_energy(Ub, COARSE[1])),
                     ("ek_fine", ek_f), ("dek_fine", dek_f), ("dek_coarse_filtered", dek_c)):
            rec[k].append(v)
        if keep_state_at is not None and any(abs(t - tk) < 1e-9 for tk in keep_state_at):
            states[f"U_{t:.3f}"] = Ub.astype(np.float32)
        extra = ""
        if not reference:
            nuc = rec["nu_closure"][-1]
            extra = (f" | closure-term fit mean {nuc.mean() / NU_SCALE:.3f} zero frac {(nuc == 0).mean():.2f}")
        _save_gen(out, ic, rec, states)  # after every snapshot, so a cut-off run keeps its data
        log(f"[gen {ic}] t={t:.3f} Ek fine {ek_f:.6f} filtered {rec['ek_filtered'][-1]:.6f} "
            f"eps fine {-dek_f:.5f} nu_t/mu mean {nut.mean() / NU_SCALE:.3f} max {nut.max() / NU_SCALE:.2f} "
            f"zero frac {(nut == 0).mean():.2f}{extra} ({time.time() - t0:.0f} s)")
    gf.close()
    gc.close()
    log(f"[gen {ic}] wrote {out}")


def _save_gen(out, ic, rec, states):
    np.savez_compressed(out, ic=ic, fine=np.array(FINE), coarse=np.array(COARSE), t=np.array(rec["t"]),
                        nut=np.array(rec["nut"]), feats=np.array(rec["feats"], dtype=np.float32),
                        ek_filtered=np.array(rec["ek_filtered"]), ek_fine=np.array(rec["ek_fine"]),
                        dek_fine=np.array(rec["dek_fine"]), dek_coarse_filtered=np.array(rec["dek_coarse_filtered"]),
                        nu_closure=np.array(rec.get("nu_closure", [])), **states)


# ------------------------------------------------------------------------------------------
# train
# ------------------------------------------------------------------------------------------
def _pairs(paths, skip_t0=True):
    X, y = [], []
    for pth in paths:
        d = np.load(pth)
        for s in range(len(d["t"])):
            if skip_t0 and d["t"][s] == 0.0:
                continue
            X.append(d["feats"][s])
            y.append(d["nut"][s] / NU_SCALE)
    return np.concatenate(X).astype(np.float32), np.concatenate(y).astype(np.float32)


def _init_params(F: int, seed: int) -> np.ndarray:
    """Seeded uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) initialisation (float32, flat layout)."""
    H = 64
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, size in ((F, H * F), (F, H), (H, H * H), (H, H), (H, H), (H, 1)):
        lim = 1.0 / np.sqrt(fan_in)
        parts.append(rng.uniform(-lim, lim, size))
    return np.concatenate(parts).astype(np.float32)


def train_model(data, val, out, epochs=300, batch=4096, lr=1e-3, seed=0):
    import torch

    fr = _fr()
    X, y = _pairs(data)
    Xv, yv = _pairs(val)
    F = X.shape[1]
    mean = X.mean(axis=0)
    std = X.std(axis=0) + 1e-3
    net = fr.MLP(F, _init_params(F, seed), mean, std)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    Xvd, yvd = torch.from_numpy(Xv).cuda(), torch.from_numpy(yv).cuda()
    gen_ = torch.Generator(device="cuda")
    gen_.manual_seed(seed)
    n = X.shape[0]
    batch = min(batch, n)
    hist = []
    base_tr = float(np.mean((y - y.mean()) ** 2))
    base_va = float(np.mean((yv - y.mean()) ** 2))
    t0 = time.time()
    for ep in range(epochs):
        lr_ep = lr * (0.5 * (1 + np.cos(np.pi * ep / epochs)) * 0.9 + 0.1)
        perm = torch.randperm(n, device="cuda", generator=gen_)
        for b in range(0, n - batch + 1, batch):
            idx = perm[b:b + batch]
            net.train_step(Xd[idx].contiguous(), yd[idx].contiguous(), lr_ep)
        if ep % 20 == 0 or ep == epochs - 1:
            ltr, _ = net.loss_grad(Xd, yd)
            lva, _ = net.loss_grad(Xvd, yvd)
            hist.append((ep, ltr, lva))
            log(f"[train] epoch {ep} lr {lr_ep:.2e} loss train {ltr:.4f} val {lva:.4f} "
                f"(constant predictor: {base_tr:.4f} / {base_va:.4f}) {time.time() - t0:.1f} s")
    params = net.get_params()
    net.close()
    np.savez(out, params=params, mean=mean.astype(np.float32), std=std.astype(np.float32), n_in=F,
             nu_scale=NU_SCALE, prandtl_t=PRANDTL_T, history=np.array(hist), base_train=base_tr, base_val=base_va,
             n_train=n, n_val=Xv.shape[0])
    log(f"[train] wrote {out}")


# ------------------------------------------------------------------------------------------
# eval: a-posteriori comparison on the coarse mesh
# ------------------------------------------------------------------------------------------
def spectrum(U: np.ndarray, shape, p: int):
    """Shell-summed kinetic-energy spectrum of the velocity of a state on an uncurved periodic
    box, from its values interpolated to n_e (p+1) equispaced points per direction."""
    n = p + 1
    xs = np.polynomial.legendre.leggauss(n)[0]
    xe = -1.0 + (2 * np.arange(n) + 1.0) / n
    L = np.stack([np.prod([(xe - xs[m]) / (xs[b] - xs[m]) for m in range(n) if m != b], axis=0)
                  for b in range(n)], axis=1)  # [equispaced][gauss]
    nx, ny, nz = shape
    vel = U[:, 1:4] / U[:, 0:1]
    T = vel.reshape(nz, ny, nx, 3, n, n, n)                       # ke je ie c k j i
    T = np.einsum("ai,zyxckji->zyxckja", L, T)
    T = np.einsum("bj,zyxckja->zyxckba", L, T)
    T = np.einsum("ck,zyxdkba->zyxdcba", L, T)
    G = np.transpose(T, (3, 0, 4, 1, 5, 2, 6)).reshape(3, nz * n, ny * n, nx * n)
    N = G.shape[1]
    uh = np.fft.fftn(G, axes=(1, 2, 3)) / N ** 3
    e = 0.5 * (np.abs(uh) ** 2).sum(axis=0)
    k = np.fft.fftfreq(N, 1.0 / N)
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    kk = np.rint(np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)).astype(int)
    return np.bincount(kk.ravel(), weights=e.ravel())[: N // 2 + 1]


def coarse_run(model_path, ref_t, state_times=()):
    """E_k and dE_k/dt of the coarse TGV run at the reference times, with or without the model."""
    fr = _fr()
    _, mc = meshes()
    g = fr.FRMesh(mc, COARSE[1], mu=MU, flux=FLUX, check_finite=True)
    g.set_state(make_state("tgv", mc, g))
    net = None
    if model_path:
        d = np.load(model_path)
        net = fr.MLP(int(d["n_in"]), d["params"], d["mean"], d["std"])
        g.set_sgs_model(net, float(d["nu_scale"]), float(d["prandtl_t"]))
    ek, dek, states, nut_mean = [], [], {}, []
    t = 0.0
    for tk in ref_t:
        nsteps = int(round((tk - t) / DT_COARSE))
        if nsteps > 0:
            g.rk_step(DT_COARSE, "lsrk45", nsteps)
        t = tk
        a, b = g.kinetic_energy()
        ek.append(a)
        dek.append(b)
        if net is not None:
            nut_mean.append(float(g.eddy_viscosity().mean()))
        if any(abs(t - s) < 1e-9 for s in state_times):
            states[t] = g.get_state()
    g.close()
    if net is not None:
        net.close()
    return np.array(ek), np.array(dek), states, np.array(nut_mean)


def evaluate(model_path, ref_path, out=None):
    ref = np.load(ref_path)
    t = ref["t"]
    ek_ref = ref["ek_filtered"]
    # dissipation rate of the filtered reference by central differences (one-sided at the ends)
    eps_ref = -np.gradient(ek_ref, t)
    t_end = float(t[-1])
    res = {}
    for name, mp in (("implicit_les", None), ("learned_closure", model_path)):
        ek, dek, states, nut = coarse_run(mp, t, state_times=(t_end,))
        e_ek = float(np.sqrt(np.mean((ek - ek_ref) ** 2)) / np.mean(ek_ref))
        e_eps = float(np.sqrt(np.mean((-dek - eps_ref) ** 2)) / np.max(np.abs(eps_ref)))
        res[name] = {"ek": ek.tolist(), "eps": (-dek).tolist(), "rel_l2_ek": e_ek, "rel_l2_eps": e_eps,
                     "nu_t_over_mu_mean": (nut / NU_SCALE).tolist() if nut.size else None}
        if f"U_{t_end:.3f}" in ref.files:
            sr = spectrum(ref[f"U_{t_end:.3f}"].astype(np.float64), (COARSE[0],) * 3, COARSE[1])
            sl = spectrum(states[t_end], (COARSE[0],) * 3, COARSE[1])
            kmax = COARSE[0] * (COARSE[1] + 1) // 3  # compare up to a third of the grid's wavenumbers
            a, b = sl[1:kmax + 1], sr[1:kmax + 1]
            ok = (b > 1e-10 * sr.max()) & (a > 0)  # wavenumbers that carry energy
            res[name]["spectrum_rel_err"] = float(np.sqrt(np.mean((np.log(a[ok]) - np.log(b[ok])) ** 2)))
            res[name]["spectrum"] = sl[: kmax + 1].tolist()
            res["spectrum_ref"] = sr[: kmax + 1].tolist()
        log(f"[eval] {name}: rel L2 error E_k {e_ek:.4g}, dissipation rate {e_eps:.4g}"
            + (f", log-spectrum rms {res[name]['spectrum_rel_err']:.4g}" if "spectrum_rel_err" in res[name] else ""))
    res["t"] = t.tolist()
    res["ek_ref"] = ek_ref.tolist()
    res["eps_ref"] = eps_ref.tolist()
    res["gain_ek"] = res["implicit_les"]["rel_l2_ek"] / res["learned_closure"]["rel_l2_ek"]
    res["gain_eps"] = res["implicit_les"]["rel_l2_eps"] / res["learned_closure"]["rel_l2_eps"]
    log(f"[eval] error ratio (implicit LES / learned closure): E_k {res['gain_ek']:.3f}, "
        f"dissipation rate {res['gain_eps']:.3f}")
    if out:
        with open(out, "w") as f:
            json.dump(res, f, indent=1)
    return res


def scale_check(t_end: float, every: float, out: str, dt_fine=None, dt_coarse=None):
    """Implicit LES at the coarse resolution against the fine run: the TGV at both (no closure),
    the fine run's energy filtered to the coarse space and its dissipation rate, the coarse run's
    energy and dissipation rate at the same times. Where the coarse run dissipates more than the
    fine one, a positive eddy viscosity adds to an excess."""
    global DT_FINE, DT_COARSE
    if dt_fine:
        DT_FINE = dt_fine
    if dt_coarse:
        DT_COARSE = dt_coarse
    ref_path = out + ".ref.npz"
    gen("tgv", t_end, every, ref_path, reference=True)
    ref = np.load(ref_path)
    t = ref["t"]
    ek, dek, _, _ = coarse_run(None, t)
    res = {"fine": list(FINE), "coarse": list(COARSE), "dt_fine": DT_FINE, "dt_coarse": DT_COARSE,
           "t": t.tolist(), "ek_filtered": ref["ek_filtered"].tolist(), "eps_fine": (-ref["dek_fine"]).tolist(),
           "ek_coarse": ek.tolist(), "eps_coarse": (-dek).tolist()}
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    for i in range(len(t)):
        log(f"t={t[i]:.2f} E_k filtered fine {res['ek_filtered'][i]:.6f} coarse {ek[i]:.6f} | "
            f"eps fine {res['eps_fine'][i]:.5f} coarse {-dek[i]:.5f}")
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2308_06605_amd.closure")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("gen")
    a.add_argument("--ic", required=True)
    a.add_argument("--t-end", type=float, required=True)
    a.add_argument("--every", type=float, default=0.25)
    a.add_argument("--keep-state-at", type=float, nargs="*", default=None)
    a.add_argument("--out", required=True)
    b = sub.add_parser("train")
    b.add_argument("--data", nargs="+", required=True)
    b.add_argument("--val", nargs="+", required=True)
    b.add_argument("--epochs", type=int, default=300)
    b.add_argument("--lr", type=float, default=1e-3)
    b.add_argument("--out", required=True)
    c = sub.add_parser("eval")
    c.add_argument("--model", required=True)
    c.add_argument("--ref", required=True)
    c.add_argument("--out", default=None)
    s = sub.add_parser("scale", help="implicit LES at the coarse resolution against the fine run")
    s.add_argument("--t-end", type=float, default=7.0)
    s.add_argument("--every", type=float, default=0.5)
    s.add_argument("--dt-fine", type=float, default=None)
    s.add_argument("--dt-coarse", type=float, default=None)
    s.add_argument("--out", required=True)
    for q in (a, b, c, s):
        q.add_argument("--fine", type=int, nargs=2, default=None, metavar=("N", "P"))
        q.add_argument("--coarse", type=int, nargs=2, default=None, metavar=("N", "P"))
    a.add_argument("--reference", action="store_true", help="filtered energies only (no targets)")
    args = ap.parse_args(argv)
    configure(args.fine, args.coarse)
    if args.cmd == "gen":
        gen(args.ic, args.t_end, args.every, args.out, args.keep_state_at, args.reference)
    elif args.cmd == "scale":
        scale_check(args.t_end, args.every, args.out, args.dt_fine, args.dt_coarse)
    elif args.cmd == "train":
        train_model(args.data, args.val, args.out, epochs=args.epochs, lr=args.lr)
    else:
        evaluate(args.model, args.ref, args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
