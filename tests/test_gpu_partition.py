"""A mesh split into parts that exchange their shared faces once per stage, on one GPU
(fr_part_*; the one-GPU form of the paper's per-process run with a face exchange after the
pre-pass, sections "Pre-processor Parallelization" and "Three-level Parallelization Design").

Every part's face buffer gets the other parts' sides of the shared faces through the pack and
unpack kernels; both parts of a shared face then compute its common flux from the same data, so
the residual and every RK step must equal the unsplit mesh's bit for bit.
"""
import numpy as np
import pytest

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


def _zslab(n, nparts):
    k = np.arange(n ** 3) // (n * n)
    return (k * nparts // n).astype(np.int32)


def _compare(fr, m, p, part, U, steps, kw, fuse=True, tiles=None):
    g = fr.FRMesh(m, p, **kw)
    grp = fr.PartitionGroup(m, p, part, **kw)
    for mesh in [g, *grp.parts]:
        mesh.set_fusion(fuse)
        if tiles is not None:
            mesh.set_tiles(*tiles)
    g.set_state(U)
    grp.set_state(U)
    R0, R1 = g.residual(), grp.residual()
    assert np.array_equal(R0, R1), np.abs(R0 - R1).max()
    for scheme, dt, n in steps:
        g.rk_step(dt, scheme, n)
        grp.rk_step(dt, scheme, n)
        U0, U1 = g.get_state(), grp.get_state()
        assert np.isfinite(U0).all()
        assert np.array_equal(U0, U1), (scheme, np.abs(U0 - U1).max())
    g.close()
    grp.close()


@pytest.mark.parametrize("fuse", [True, False])
def test_two_slabs_match_the_unsplit_mesh(fuse):
    """16^3 curved box, p=3, Roe + BR2, cut into two z-slabs: residual, LSRK45, RK4 and SSP steps."""
    fr = _fr()
    n, p = 16, 3
    m = I.box_mesh(n, q=3, curve_amp=0.05)
    X = fr.FRMesh(m, p).sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=7, amp=0.02)
    print(f"16^3 p=3 two slabs, fuse={fuse}", flush=True)
    _compare(fr, m, p, _zslab(n, 2), U, [("lsrk45", 2.5e-4, 3), ("rk4", 2.5e-4, 1), ("ssprk104", 2.5e-4, 1)],
             dict(mu=MU, flux="roe"), fuse=fuse)


def test_two_slabs_fp32_form():
    fr = _fr()
    n, p = 12, 3
    m = I.box_mesh(n, q=3, curve_amp=0.05)
    X = fr.FRMesh(m, p).sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=8, amp=0.02)
    print("12^3 p=3 two slabs, FP32 form", flush=True)
    _compare(fr, m, p, _zslab(n, 2), U, [("lsrk45", 2.5e-4, 2)],
             dict(mu=MU, flux="roe", prec="fp32", ref_rho=1.0, ref_p=P0))


@pytest.mark.parametrize("p,prec", [(2, "fp64"), (5, "fp64"), (7, "fp32")])
def test_random_three_part_map_on_a_scrambled_mesh(p, prec):
    """An arbitrary element -> part map on a relabelled, rotated curved mesh: parts are not
    contiguous, faces are shared in every orientation and with either side as the owner."""
    fr = _fr()
    m = I.box_mesh(4, q=min(p, 3), curve_amp=0.05, curve_mode="mixed")
    m, _ = I.scramble_mesh(m, seed=p)
    part = np.random.default_rng(p).integers(0, 3, size=m.n_elem).astype(np.int32)
    X = fr.FRMesh(m, p).sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=p, amp=0.02)
    kw = dict(mu=MU, flux="rusanov")
    if prec == "fp32":
        kw.update(prec="fp32", ref_rho=1.0, ref_p=P0)
    print(f"4^3 p={p} {prec} random three-part map", flush=True)
    _compare(fr, m, p, part, U, [("lsrk45", 1e-4, 2)], kw, tiles=(1, 1))


def test_channel_with_walls_in_both_parts():
    """Walls belong to the part of their element; the split runs along the channel's periodic x
    direction, so both parts have walls."""
    fr = _fr()
    n = 6
    m = I.box_mesh(n, q=2, periodic=(True, False, True), curve_amp=0.05, curve_mode="mixed")
    tags = I.boundary_tags(m)
    kw = dict(mu=MU, flux="roe", bc_tag=tags, wall_T=P0)
    X = fr.FRMesh(m, 3, **kw).sol_coords()
    U = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=3, amp=0.01)
    part = (np.arange(m.n_elem) % n >= n // 2).astype(np.int32)
    print("channel with walls, split along x", flush=True)
    _compare(fr, m, 3, part, U, [("lsrk45", 1e-4, 2)], kw)


def test_halo_messages_and_refusals():
    """Message sizes from the layout, a pack/unpack round trip through the Python API, and the
    single-mesh calls a part refuses."""
    import torch

    fr = _fr()
    n, p = 8, 3
    m = I.box_mesh(n, q=1)
    grp = fr.PartitionGroup(m, p, _zslab(n, 2), mu=MU, flux="roe")
    X = fr.FRMesh(m, p).sol_coords()
    U = I.state_from_coords(X, I.tgv_state)
    grp.set_state(U)
    R = grp.residual()
    nf, nb = grp.halo_size(0, 1)
    assert nf == 2 * n * n and nb == nf * 20 * (p + 1) ** 2 * 8
    # re-sending part 0's current face data to part 1 changes nothing
    buf = torch.empty(nb // 8, dtype=torch.float64, device="cuda")
    grp.halo_pack(0, 1, buf)
    grp.halo_unpack(1, 0, buf)
    assert torch.isfinite(buf).all()
    assert np.array_equal(grp.residual(), R)
    with pytest.raises(ValueError):
        grp.halo_pack(0, 1, buf[:10])
    with pytest.raises(fr.FRError) as ei:
        grp.parts[0].residual()
    assert ei.value.name == "FR_ERR_UNSUPPORTED"
    with pytest.raises(fr.FRError):
        grp.parts[0].rk_step(1e-4)
    # fr_mesh_destroy refuses a part: the group owns it
    assert fr.load().fr_mesh_destroy(grp.parts[0].h) == -1
    grp.close()
    # LDG would need a second exchange per stage: refused
    import ctypes

    keep = []
    d = fr._desc(m, p, MU, 1.4, 0.72, 6.0, "roe", "fp64", False, keep, viscous="ldg")
    h = ctypes.c_void_p()
    part = _zslab(n, 2)
    rc = fr.load().fr_part_create(ctypes.byref(d), part.ctypes.data, 2, None, ctypes.byref(h))
    assert rc == -5 and not h.value
