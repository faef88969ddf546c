"""GPU: the learned-guess network and its kernels (C ABI) against the numpy
oracle, and the guess inside the time step.

Tolerances.  GPU and oracle round to BF16 at the same tensor boundaries, but
their FP32 sums (MFMA order vs an exact FP64 sum rounded once) differ by a
few FP32 ulps, so a hidden activation whose value lies within that distance
of a BF16 rounding boundary rounds differently: about 1e-4 of the entries,
each off by one BF16 ulp (2^-8 relative).  Hence:
  * features: equal except such single-ulp flips (at most 1e-3 of entries);
  * network output and gradients: 2e-3 relative in the 2-norm per tensor;
  * Adam on given gradients: FP32 arithmetic in the same order, 2e-6 relative;
  * the time step from a guess: the guess enters the FP64 Krylov solve as data,
    so GPU and oracle started from the GPU's guess agree to the per-step bar
    (1e-10) with identical iteration counts.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import Oracle
from oracle import guess_net as G

pytestmark = pytest.mark.gpu

FIELDS = ("phi_p", "phi_n", "mu_p", "mu_n")


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_03575_amd import library
    library()


def case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def cuda(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def state_to_grid(s, H, W):
    s = np.asarray(s)
    n = H * W
    return G.fields_grid(s[0:2 * n:2], s[1:2 * n:2], s[2 * n::2], s[2 * n + 1::2], H, W)


def grid_to_state(g):
    n = g.shape[1] * g.shape[2]
    s = np.zeros(4 * n)
    s[0:2 * n:2], s[1:2 * n:2] = g[0].ravel(), g[1].ravel()
    s[2 * n::2], s[2 * n + 1::2] = g[2].ravel(), g[3].ravel()
    return s


def smooth_states(H, W, seed=1):
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.linspace(0, 1, H), np.linspace(0, 1, W), indexing="ij")
    base = np.stack([0.1 + 0.02 * np.sin(3 * xx + k) * np.cos(2 * yy) for k in range(4)])
    base[2:] *= 30.0   # chemical potentials have a larger scale
    x2 = base + 1e-3 * rng.standard_normal(base.shape)
    x1 = x2 + 1e-4 * (np.cos(5 * xx + yy)[None] + 0.1 * rng.standard_normal(base.shape))
    x0 = x1 + 1.1 * (x1 - x2) + 1e-6 * rng.standard_normal(base.shape)
    return x2, x1, x0


def make_net(max_px, params):
    from paper_2204_03575_amd import Net
    net = Net(max_px)
    net.set_params(params)
    return net


def rand_params(seed=3):
    return S.net_init(seed=seed, zero_last=False, bias_scale=0.1)


# ---------------------------------------------------------------- network kernels
@pytest.mark.parametrize("shape", [(2, 37, 29), (1, 2, 2), (3, 5, 70), (1, 257, 257)],
                         ids=lambda s: "x".join(map(str, s)))
def test_forward_matches_oracle(shape):
    case("net forward", shape=shape)
    B, h, w = shape
    params = rand_params()
    rng = np.random.default_rng(sum(shape))
    feats = G.bf16(rng.standard_normal((B, h, w, 8)).astype(np.float32))
    net = make_net(B * h * w, params)
    y = net.forward(cuda(feats)).cpu().numpy()
    _, yo = G.forward(params, feats)
    e = rel(y, yo)
    print("relative difference of the output:", e, flush=True)
    assert e <= 2e-3


def test_gradients_match_oracle():
    case("net gradients 2x20x23 with a mask")
    params = rand_params(5)
    rng = np.random.default_rng(21)
    B, h, w = 2, 20, 23
    feats = G.bf16(rng.standard_normal((B, h, w, 8)).astype(np.float32))
    tgt = rng.standard_normal((B, h, w, 4)).astype(np.float32)
    mask = np.stack([G.crop_mask(40, 40, 3, 5, h, w), G.crop_mask(40, 40, 0, 0, h, w)]).astype(np.uint8)
    wts = np.array([1.7, 0.6])
    net = make_net(B * h * w, params)
    grads, loss = net.gradients(cuda(feats), cuda(tgt), cuda(mask), wts, smooth=3.0)
    acts, yo = G.forward(params, feats)
    lo, gy = G.loss_and_grad_output(yo, tgt, mask, wts, smooth=3.0)
    go = G.backward(params, acts, gy)
    print("loss", loss, lo, flush=True)
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    for k in range(4):
        for j, name in enumerate(("w", "b")):
            e = rel(grads[k][j], go[k][j])
            print(f"layer {k} d{name}: relative difference {e:.2e}", flush=True)
            assert e <= 2e-3, (k, name, e)


def test_adam_matches_oracle():
    case("adam, two steps")
    params = rand_params(7)
    rng = np.random.default_rng(8)
    grads = [(rng.standard_normal(w.shape).astype(np.float32) * 1e-2,
              rng.standard_normal(b.shape).astype(np.float32) * 1e-2) for w, b in params]
    net = make_net(16, params)
    m = G.zeros_like_params(params)
    v = G.zeros_like_params(params)
    po = params
    for t in (1, 2):
        net.adam(grads, 1e-3)
        po, m, v = G.adam(po, grads, m, v, t, 1e-3)
    got = net.get_params()
    for k in range(4):
        for j in range(2):
            assert np.allclose(got[k][j], po[k][j], rtol=2e-6, atol=1e-9), (k, j)


def test_params_round_trip_and_zero_last_layer_is_linear_extrapolation():
    case("params round trip; zero last layer")
    import torch
    params = S.net_init(seed=11, zero_last=True)
    H, W = 17, 13
    net = make_net(H * W, params)
    got = net.get_params()
    for k in range(4):
        assert np.array_equal(got[k][0], params[k][0]) and np.array_equal(got[k][1], params[k][1])
    x2, x1, _ = smooth_states(H, W)
    s2, s1 = cuda(grid_to_state(x2)), cuda(grid_to_state(x1))
    g = net.guess(H, W, s2, s1).cpu().numpy()
    s1h, s2h = s1.cpu().numpy(), s2.cpu().numpy()
    assert np.array_equal(g, s1h + (s1h - s2h))
    del torch


# ---------------------------------------------------------------- features and guess
@pytest.mark.parametrize("HW", [(17, 13), (2, 2), (65, 65)], ids=lambda s: "x".join(map(str, s)))
def test_features_and_guess_match_oracle(HW):
    case("features and guess", HW=HW)
    H, W = HW
    x2, x1, _ = smooth_states(H, W, seed=H)
    params = rand_params(13)
    net = make_net(H * W, params)
    s2, s1 = cuda(grid_to_state(x2)), cuda(grid_to_state(x1))
    feats, sigma = net.features(H, W, s2, s1)
    fo, so = G.features(x2, x1)
    feats = feats.cpu().numpy()
    assert np.allclose(sigma, so, rtol=1e-13, atol=0)
    diff = feats != fo
    print("feature entries that differ:", int(diff.sum()), "of", diff.size, flush=True)
    assert diff.mean() <= 1e-3
    if diff.any():   # only single-ulp BF16 flips
        assert np.all(np.abs(feats[diff] - fo[diff]) <= 2.0 ** -7 * np.abs(fo[diff]) + 1e-30)
    g = state_to_grid(net.guess(H, W, s2, s1).cpu().numpy(), H, W)
    _, yo = G.forward(params, fo[None])
    go = G.guess(x2, x1, yo[0], so)
    corr = go - (2 * x1 - x2)
    e = np.linalg.norm(g - go) / max(np.linalg.norm(corr), 1e-300)
    print("guess: difference relative to the learned correction", e, flush=True)
    assert e <= 2e-3


# ---------------------------------------------------------------- the guess inside the step
def oracle_step_from(o, php, phn, start, rtol):
    """The oracle's FGMRES for both species from the given start state vector."""
    b = o.rhs(php, phn)
    n = php.size
    out = {}
    its = []
    for s, (ph, mu) in enumerate((("phi_p", "mu_p"), ("phi_n", "mu_n"))):
        x0 = np.concatenate([start[s:2 * n:2], start[2 * n + s::2]])
        x, it, rr = o.fgmres(s, b[s], x0)
        out[ph], out[mu] = x[:n], x[n:]
        its.append(it)
    return out, tuple(its)


def residual_norms(o, php, phn, state):
    """Per species: the residual's 2-norm, the norm of b, and the residual norm
    of the first block row (the one the start choice ranks by)."""
    b = o.rhs(php, phn)
    n = php.size
    rs = [b[s] - o.apply_saddle(s, np.concatenate([state[s:2 * n:2], state[2 * n + s::2]]))
          for s in range(2)]
    return ([np.linalg.norm(r) for r in rs], [np.linalg.norm(b[s]) for s in range(2)],
            [np.linalg.norm(r[:n]) for r in rs])


@pytest.mark.parametrize("mode,evap", [("linear", 0.0), ("learned", 0.0), ("linear", 0.003),
                                       ("learned", 0.003)])
def test_step_with_guess_matches_oracle(mode, evap):
    case("step with guess", mode=mode, evap=evap)
    from paper_2204_03575_amd import Solver
    p = S.preset("square32", n=(24, 20), evap_ds=evap, evap_steps=100)
    co, ce = S.make_mesh(p)
    H, W = 21, 25
    n = co.shape[0]
    g = Solver(co, ce, p)
    o = Oracle(co, ce, p)
    php, phn, _ = S.initial_fractions(n, p["mean_p"], p["mean_n"])
    g.set_fields(php, phn)
    g.step(1)                         # history: the solutions of two steps
    y2 = g.get_state(solution=True).cpu().numpy()
    g.step(1)
    net = None
    if mode == "learned":
        net = make_net(H * W, S.net_init(seed=17, zero_last=False, bias_scale=0.01))
    g.set_guess(mode, net, H, W)
    chosen = []
    for k in range(4):
        x1 = g.get_state().cpu().numpy()               # the state the step starts from
        y1 = g.get_state(solution=True).cpu().numpy()  # the last solution
        if evap == 0.0:
            assert np.array_equal(x1, y1)
        cur = g.get_fields()
        stats = g.step(1)[0]
        got = g.get_fields()
        cands = [x1, y1 + (y1 - y2)]
        if mode == "learned":
            cands.append(net.guess(H, W, cuda(y2), cuda(y1)).cpu().numpy())
        norms = [residual_norms(o, cur["phi_p"], cur["phi_n"], c) for c in cands]
        res = [nm[0] for nm in norms]
        first = [nm[2] for nm in norms]
        bn = norms[0][1]
        start = x1.copy()
        for s in range(2):
            want = int(np.argmin([r[s] for r in first]))   # first minimum: ties keep the simpler
            assert stats["guess_used"][s] == want, (k, s, res, stats)
            assert abs(stats["res0"][s] - res[want][s] / bn[s]) <= 1e-10 * res[want][s] / bn[s]
            chosen.append(want)
            c = cands[want]
            start[s:2 * n:2], start[2 * n + s::2] = c[s:2 * n:2], c[2 * n + s::2]
        ref, its = oracle_step_from(o, cur["phi_p"], cur["phi_n"], start, p["rtol"])
        if evap > 0.0:   # the step removes solvent after the solve, as the oracle's step does
            sp, sn = ref["phi_p"], ref["phi_n"]
            tot = sp + sn
            ref["phi_p"], ref["phi_n"] = sp + evap * sp / tot, sn + evap * sn / tot
        print(f"step {k}: {stats}; oracle iterations {its}; residuals {res}", flush=True)
        assert stats["iters"] == its
        for f in FIELDS:
            assert rel(got[f], ref[f]) <= 1e-10, (k, f, rel(got[f], ref[f]))
        y2 = y1
    assert max(chosen) > 0   # extrapolating the solutions beats the previous state here
    del net


def test_bad_network_falls_back_to_extrapolation():
    case("fallback: a network with a huge output")
    from paper_2204_03575_amd import Solver
    p = S.preset("square32", n=(16, 16))
    co, ce = S.make_mesh(p)
    params = S.net_init(seed=19, zero_last=False, bias_scale=0.0)
    params[-1] = (params[-1][0], np.full(4, 1e6, np.float32))   # output bias 1e6 sigma
    net = make_net(17 * 17, params)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    runs = []
    for mode in ("linear", "learned"):
        g = Solver(co, ce, p)
        g.set_fields(php, phn)
        g.set_guess(mode, net if mode == "learned" else None, 17, 17)
        st = g.step(5)
        runs.append((st, g.get_fields()))
        del g
    for a, b in zip(runs[0][0], runs[1][0]):
        assert a["iters"] == b["iters"] and a["guess_used"] == b["guess_used"]
        assert 2 not in b["guess_used"]
    for f in FIELDS:
        assert np.array_equal(runs[0][1][f], runs[1][1][f])


def test_train_step_matches_oracle():
    case("one training step on three crops")
    H, W, ch, cw = 20, 22, 12, 13
    trip = [smooth_states(H, W, seed=s) for s in (31, 32, 33)]
    oy, ox = np.array([0, 8, 3]), np.array([9, 0, 4])
    params = S.net_init(seed=23, zero_last=False, bias_scale=0.05)
    net = make_net(3 * ch * cw, params)
    x2s = [cuda(grid_to_state(t[0])) for t in trip]
    x1s = [cuda(grid_to_state(t[1])) for t in trip]
    x0s = [cuda(grid_to_state(t[2])) for t in trip]
    lr = 1e-3
    loss = net.train_step(H, W, ch, cw, x2s, x1s, x0s, oy, ox, lr, smooth=2.0)
    feats, tgts, masks, wts = [], [], [], []
    for (x2, x1, x0), a, b in zip(trip, oy, ox):
        f, sg = G.features(x2, x1)
        t = G.target(x2, x1, x0, sg)
        feats.append(f[a:a + ch, b:b + cw])
        tgts.append(t[a:a + ch, b:b + cw])
        masks.append(G.crop_mask(H, W, a, b, ch, cw))
        wts.append(G.sample_weight(x2, x1, x0, sg))
    feats, tgts, masks = np.stack(feats), np.stack(tgts), np.stack(masks)
    acts, yo = G.forward(params, feats)
    lo, gy = G.loss_and_grad_output(yo, tgts, masks, wts, smooth=2.0)
    go = G.backward(params, acts, gy)
    po, _, _ = G.adam(params, go, G.zeros_like_params(params), G.zeros_like_params(params), 1, lr)
    print("loss", loss, lo, "weights", wts, flush=True)
    assert abs(loss - lo) <= 1e-4 * abs(lo)
    got = net.get_params()
    for k in range(4):
        for j in range(2):
            du = (got[k][j] - params[k][j]).astype(np.float64)
            do = (po[k][j] - params[k][j]).astype(np.float64)
            off = np.abs(du - do) > 1e-2 * lr
            print(f"layer {k} {'wb'[j]}: updates off by more than lr/100: {int(off.sum())} of {off.size}",
                  flush=True)
            assert np.all(np.abs(du - do) <= 2.0 * lr + 1e-9)
            assert off.mean() <= 0.02


def test_set_guess_rejects_bad_arguments():
    case("chm_set_guess argument checks")
    from paper_2204_03575_amd import ChmError, Solver
    p = S.preset("square32", n=(8, 8))
    co, ce = S.make_mesh(p)
    g = Solver(co, ce, p)
    net = make_net(81, S.net_init())
    with pytest.raises(ChmError):
        g.set_guess("learned", None, 9, 9)
    with pytest.raises(ChmError):
        g.set_guess("learned", net, 9, 8)         # H * W != vertices
    small = make_net(16, S.net_init())
    with pytest.raises(ChmError):
        g.set_guess("learned", small, 9, 9)       # grid larger than max_pixels
    g.set_guess("learned", net, 9, 9)
    g.set_guess("previous")


def test_trained_network_gains_over_the_previous_state_start():
    """The committed network (trained on 256x256 runs) on a run outside its
    training set: fewer FGMRES iterations than starting every solve from the
    previous state (the method without a guess); linear extrapolation, which
    the learned mode also offers, is reported beside it."""
    case("trained network, 256x256, 60 steps of a held-out run")
    import os
    from paper_2204_03575_amd import Net, Solver
    from paper_2204_03575_amd import guess_train as T
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    params = np.load(os.path.join(root, "paper_2204_03575_amd", "weights", "guess256.npy"))
    n, H = 256, 257
    p, seed = T.run_params(n, 1001, 20220500)
    co, ce = S.make_mesh(p)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"], seed=seed)
    net = Net(H * H)
    net.set_params(params)
    iters = {}
    for mode in ("previous", "linear", "learned"):
        g = Solver(co, ce, p)
        g.set_fields(php, phn)
        g.set_guess(mode, net if mode == "learned" else None, H, H)
        st = g.step(60)
        iters[mode] = float(np.mean([s["iters"] for s in st]))
        assert max(max(s["relres"]) for s in st) <= p["rtol"]
        del g
    print("mean FGMRES iterations per species and step:", iters, flush=True)
    assert iters["learned"] < iters["previous"]
