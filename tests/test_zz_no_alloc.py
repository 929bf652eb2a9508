"""csi_mlp_forward_noalloc (the library's own per-GPU scratch, no work
argument) against csi_mlp_forward (caller's work buffer) through the C-ABI:
the same kernels on the same packed operands, so the outputs are bitwise
equal; and both against the numpy BF16-emulating oracle.  Two calls in a row,
the second with a smaller network and fewer samples, so that stale scratch
contents of the first call would show."""
import numpy as np
import pytest

from oracle import mlp
from paper_2403_03440_amd import inputs as I

pytestmark = pytest.mark.gpu


def _case(n_in, n_out, n, seed):
    p = mlp.init_params(n_in, n_out, I.uniform_pm1(seed, mlp.n_params(n_in, n_out)))
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p, n_in, n_out)
    b1[:] = 0.1 * I.uniform_pm1(seed + 1, b1.size)
    b3[:] = 0.1 * I.uniform_pm1(seed + 3, b3.size)
    p = mlp.pack(W1, b1, W2, b2, W3, b3).astype(np.float32)
    x = (2.0 * I.uniform_pm1(seed + 5, n * n_in).reshape(n, n_in)).astype(np.float32)
    return p, x


def test_forward_noalloc_matches_forward():
    import torch
    from paper_2403_03440_amd import csi
    for n_in, n_out, n, seed in ((64, 1024, 3001, 41), (14, 121, 700, 43)):
        print(f"noalloc forward n_in {n_in} n_out {n_out} n {n}", flush=True)
        p, x = _case(n_in, n_out, n, seed)
        net = csi.Mlp(n_in, n_out, batch=256)
        pd = torch.tensor(p, device="cuda")
        xd = torch.tensor(x, device="cuda")
        y_ref = net.forward(pd, xd).cpu().numpy()
        y = torch.full((n, n_out), float("nan"), dtype=torch.float32, device="cuda")
        net.forward_noalloc(pd, xd, y)
        y = y.cpu().numpy()
        assert np.array_equal(y, y_ref)
        # and against the oracle with the same rounding points (outputs away
        # from a BF16 rounding midpoint of an activation)
        p64, x64 = p.astype(np.float64), x.astype(np.float64)
        yo, (_, _, _, _, h2b) = mlp.forward(p64, x64, n_out, emulate=True)
        fb = mlp.flip_bound(p64, x64, n_out)
        W3, b3 = mlp.unpack(p64, n_in, n_out)[4:]
        scale = np.abs(h2b) @ np.abs(mlp.bf16(W3).astype(np.float64)).T + np.abs(b3)
        assert np.all(np.abs(y - yo) <= 2e-5 * scale + fb)


def test_forward_noalloc_rejects_bad_arguments():
    import torch
    from paper_2403_03440_amd import csi
    net = csi.Mlp(14, 121, batch=64)
    p, x = _case(14, 121, 10, 7)
    pd = torch.tensor(p, device="cuda")
    xd = torch.tensor(x, device="cuda")
    y = torch.empty((10, 121), dtype=torch.float32, device="cuda")
    net.n_out = 2000   # beyond the network limits: rejected before any launch
    with pytest.raises(csi.CsiError, match="CSI_ERR_ARG"):
        net.forward_noalloc(pd, xd, y)
