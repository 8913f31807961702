"""The tile autotuner: every tile choice (elements per block of the element kernels, threads per
block of the face kernel) gives the same residual and RK step bit for bit (each thread does
the same arithmetic), and the autotuner keeps the fastest choice it timed."""
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


@pytest.mark.parametrize("p,viscous,prec", [(2, "br2", "fp64"), (3, "br2", "fp64"), (3, "ldg", "fp64"),
                                            (5, "br2", "fp64"), (6, "br2", "fp64"), (2, "br2", "fp32"),
                                            (3, "br2", "fp32"), (5, "br2", "fp32"), (6, "br2", "fp32"),
                                            (7, "br2", "fp32")])
def test_tiles_bitwise_equal(p, viscous, prec):
    """Every tile choice gives the default's residual and RK steps bit for bit, on 125 elements
    (a ragged last block whenever a block holds more than one element; at p = 5 and 6 the second
    choice is two elements per block)."""
    fr = _fr()
    m = I.box_mesh(5, q=2, curve_amp=0.04)
    kw = dict(prec="fp32", ref_rho=1.0, ref_p=1.0 / (1.4 * 0.01)) if prec == "fp32" else {}
    g = fr.FRMesh(m, p, mu=1e-3, flux="roe", viscous=viscous, **kw)
    X = g.sol_coords()
    U0 = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=1, amp=0.01)
    g.set_state(U0)
    assert g.tiles() == (0, 0)
    R0 = g.residual()
    g.rk_step(1e-3, "lsrk45", 2)
    S0 = g.get_state()
    for epb in (0, 1):
        for fbs in (0, 1, 2):
            g.set_tiles(epb, fbs)
            g.set_state(U0)
            assert np.array_equal(g.residual(), R0), (epb, fbs)
            g.rk_step(1e-3, "lsrk45", 2)
            assert np.array_equal(g.get_state(), S0), (epb, fbs)
    with pytest.raises(fr.FRError):
        g.set_tiles(2, 0)
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autotune_picks_fastest(prec):
    fr = _fr()
    m = I.box_mesh(16, q=1)
    kw = dict(prec="fp32", ref_rho=1.0, ref_p=1.0 / (1.4 * 0.01)) if prec == "fp32" else {}
    g = fr.FRMesh(m, 3, mu=1e-3, flux="roe", **kw)
    g.set_state(I.state_from_coords(g.sol_coords(), I.tgv_state))
    R0 = g.residual()
    U0 = g.get_state()
    (epb, fbs), ms = g.autotune(3)
    fuse = g.fusion()
    print(prec, "tile timings (ms per stage):", ms, "chosen", (epb, fbs, fuse), flush=True)
    assert np.all(ms > 0)
    assert ms[6 * fuse + 3 * epb + fbs] == ms.min()
    # the autotuner leaves the state and every later result as they were
    assert np.array_equal(g.get_state(), U0)
    assert np.array_equal(g.residual(), R0)
    g.close()


@pytest.mark.parametrize("p,scheme,prec", [(3, "lsrk45", "fp64"), (2, "rk4", "fp64"), (7, "ssprk104", "fp64"),
                                           (3, "lsrk45", "fp32"), (6, "rk4", "fp32")])
def test_fusion_on_off_bitwise_equal(p, scheme, prec):
    """The fused pre-pass computes the same sums as the stand-alone one: stepping with fusion
    on and off gives the same states bit for bit."""
    fr = _fr()
    m = I.box_mesh(4, q=2, curve_amp=0.04)
    kw = dict(prec="fp32", ref_rho=1.0, ref_p=1.0 / (1.4 * 0.01)) if prec == "fp32" else {}
    g = fr.FRMesh(m, p, mu=1e-3, flux="roe", **kw)
    assert g.fusion()
    X = g.sol_coords()
    U0 = I.state_from_coords(X, I.tgv_state) + I.random_smooth_perturbation(X, seed=p, amp=0.01)
    out = []
    for on in (True, False):
        g.set_fusion(on)
        assert g.fusion() == on
        g.set_state(U0)
        g.rk_step(2e-4, scheme, 3)
        out.append(g.get_state())
    with pytest.raises(fr.FRError):
        fr._check(fr.load().fr_set_fusion(g.h, 2))
    g.close()
    assert np.array_equal(out[0], out[1])
