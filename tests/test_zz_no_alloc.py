"""The no-allocation entry point dsmc_mlp_backward_noalloc against the
existing dsmc_mlp_backward, through the C ABI: the same gradient bit for
bit and the same mean squared error on two calls in a row, the second with
fewer rows (the scratch keeps the first call's partials, which the second
must not read), and an error for more rows than the scratch holds."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2607_08195_amd import dsmc
    return dsmc


def test_backward_noalloc_matches_backward(D):
    import torch
    net = D.Mlp()
    net.init_weights(seed=5)
    rng = np.random.default_rng(9)
    grad = torch.empty(D.MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    for rows in (4096, 1000, 37):
        x = rng.standard_normal((rows, D.MLP_IN)).astype(np.float32)
        t = (0.1 * rng.standard_normal((rows, D.MLP_OUT))).astype(np.float32)
        l_ref, g_ref = net.backward(x, t)
        xd = torch.from_numpy(x).cuda()
        td = torch.from_numpy(t).cuda()
        grad.fill_(np.nan)
        loss.fill_(np.nan)
        torch.cuda.synchronize()
        net.backward_noalloc(xd, td, grad, loss)
        torch.cuda.synchronize()
        g = grad.cpu().numpy()
        assert np.array_equal(g, g_ref), (rows, np.abs(g - g_ref).max())
        assert float(loss.cpu()[0]) == l_ref, (rows, float(loss.cpu()[0]), l_ref)
    x = torch.zeros((4097, D.MLP_IN), dtype=torch.float32, device="cuda")
    t = torch.zeros((4097, D.MLP_OUT), dtype=torch.float32, device="cuda")
    with pytest.raises(D.DsmcError):
        net.backward_noalloc(x, t, grad, loss)
    net.close()
