"""GPU: the allocation-free guess (chm_net_guess_noalloc) against chm_net_guess.

Both run the same kernels in the same order, the first on the network's own
buffers and the second on the library's fixed device array, so the guesses
must be equal bit for bit: on two calls in a row, the second on a smaller
grid (the array keeps the first call's contents, which the second must not
depend on), with a network whose own buffers are far smaller than the grid,
and with the size limit enforced.
"""
import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_03575_amd import library
    library()


def states(H, W, seed):
    """two nearby state vectors (4 H W doubles, solver layout) on an H x W grid"""
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.linspace(0, 1, H), np.linspace(0, 1, W), indexing="ij")
    n = H * W
    base = np.zeros(4 * n)
    for c in range(4):
        f = (0.1 + 0.02 * np.sin(3 * xx + c) * np.cos(2 * yy)).ravel() * (30.0 if c >= 2 else 1.0)
        idx = (c >> 1) * 2 * n + 2 * np.arange(n) + (c & 1)
        base[idx] = f
    x2 = base + 1e-3 * rng.standard_normal(4 * n)
    x1 = x2 + 1e-4 * rng.standard_normal(4 * n)
    return x2, x1


def test_noalloc_guess_equals_guess():
    import torch

    from paper_2204_03575_amd import Net
    from paper_2204_03575_amd.chm import ChmError
    params = S.net_init(seed=11, zero_last=False, bias_scale=0.1)
    ref_net = Net(257 * 257)
    ref_net.set_params(params)
    small_net = Net(4)   # its own buffers hold 4 pixels: the array serves the grid
    small_net.set_params(params)
    for H, W, seed in ((257, 257, 1), (33, 41, 2)):
        print(f"\n[case] noalloc guess {H}x{W}", flush=True)
        x2, x1 = (torch.as_tensor(a).cuda() for a in states(H, W, seed))
        ref = ref_net.guess(H, W, x2, x1).cpu().numpy()
        out = torch.full_like(x1, float("nan"))
        small_net.guess_noalloc(H, W, x2, x1, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref)
        # linear extrapolation plus a non-zero learned correction
        assert not np.array_equal(got, (2 * x1 - x2).cpu().numpy())
    x2, x1 = (torch.as_tensor(a).cuda() for a in states(258, 257, 3))
    with pytest.raises(ChmError):
        small_net.guess_noalloc(258, 257, x2, x1, torch.empty_like(x1))
