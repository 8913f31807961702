"""The no-allocation training step (fr_mlp_train_step_noalloc) against fr_mlp_train_step.

Both calls run the same kernels on the same inputs; only where the per-sample activations,
deltas and gradient partials live differs (the library's fixed per-GPU scratch array against
the network's own buffers), so the parameters, the Adam state's effect and the loss must agree
bit for bit. Two calls in a row, the second with a smaller batch (the scratch array keeps the
first call's contents), then a batch at the maximum size and one beyond it.
"""
import ctypes

import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


def _fr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_06605_amd import fr

    fr.load()
    return fr


def _data(F, n, seed):
    rng = np.random.default_rng(seed)
    X = (rng.normal(size=(n, F)) * rng.uniform(0.5, 3, F) + rng.normal(size=F) * 4).astype(np.float32)
    t = rng.uniform(0, 4, n).astype(np.float32)
    return X, t


@pytest.mark.parametrize("F", [68, 20])
def test_noalloc_step_equals_train_step(F):
    import torch

    fr = _fr()
    X0, _ = _data(F, 4096, seed=1)
    mean = X0.mean(axis=0).astype(np.float32)
    std = (X0.std(axis=0) + 0.05).astype(np.float32)
    theta = M.init_params(F, seed=3)
    a = fr.MLP(F, theta, mean, std)
    b = fr.MLP(F, theta, mean, std)
    la = torch.zeros(1, dtype=torch.float32, device="cuda")
    lb = torch.zeros(1, dtype=torch.float32, device="cuda")
    for k, n in enumerate((5000, 700, fr.MLP_NOALLOC_MAX_N)):
        X, t = _data(F, n, seed=10 + k)
        Xd = torch.from_numpy(X).cuda()
        td = torch.from_numpy(t).cuda()
        print(f"F={F} call {k} n={n}", flush=True)
        a.train_step(Xd, td, 1e-3, loss_out=la)
        b.train_step_noalloc(Xd, td, 1e-3, loss_out=lb)
        torch.cuda.synchronize()
        pa, pb = a.get_params(), b.get_params()
        assert np.array_equal(pa.view(np.uint32), pb.view(np.uint32)), (k, np.abs(pa - pb).max())
        assert la.item() == lb.item(), (k, la.item(), lb.item())
        for wa, wb in zip(a.get_bf16(), b.get_bf16()):
            assert np.array_equal(wa, wb), k
        assert np.isfinite(la.item())
    # the same parameters predict the same values afterwards
    Xd = torch.from_numpy(_data(F, 333, seed=99)[0]).cuda()
    assert torch.equal(a.forward(Xd), b.forward(Xd))
    a.close()
    b.close()


def test_noalloc_rejects_batches_beyond_the_maximum():
    import torch

    fr = _fr()
    F = 20
    X0, _ = _data(F, 256, seed=2)
    net = fr.MLP(F, M.init_params(F, seed=4), X0.mean(axis=0), X0.std(axis=0) + 0.05)
    before = net.get_params()
    n = fr.MLP_NOALLOC_MAX_N + 1
    X = torch.zeros((n, F), dtype=torch.float32, device="cuda")
    t = torch.zeros(n, dtype=torch.float32, device="cuda")
    with pytest.raises(fr.FRError) as ei:
        net.train_step_noalloc(X, t, 1e-3)
    assert ei.value.name == "FR_ERR_ARG"
    assert "8192" in str(ei.value)
    # a rejected call leaves the network as it was
    assert np.array_equal(net.get_params(), before)
    # direct C-ABI call with n = 0 is rejected too
    rc = fr.load().fr_mlp_train_step_noalloc(net.h, ctypes.c_void_p(X.data_ptr()), 0, F,
                                             ctypes.c_void_p(t.data_ptr()), ctypes.c_float(1e-3), None)
    assert rc == -1
    net.close()
