"""Learned initial guess: plain numpy reference of the network, its training
step and the guess it makes (TEST INFRASTRUCTURE ONLY: only the tests, the
smoke check and the benchmark's CPU-baseline leg use it).

What is computed (the conventions the GPU kernels follow):

* Grid.  A 2D structured P1 mesh of (nx, ny) squares has H = ny + 1 rows and
  W = nx + 1 columns of vertices, vertex v = row * W + col.  The four fields
  phi_p, phi_n, mu_p, mu_n (channels 0..3) live on that grid.
* Features (FP64, then FP32, then BF16 round-to-nearest-even), from the
  states at steps n-2 (x2) and n-1 (x1): d = x1 - x2 with sigma_c the RMS of
  d_c over the grid, and the centred state x1_c - mean(x1_c) with tau_c its
  RMS; channels 0..3 are d_c / sigma_c, channels 4..7 the centred state
  divided by tau_c (a zero RMS gives zero features).
* Network: four 3x3 convolutions with reflective padding of one vertex (the
  discrete no-flux condition: the value beyond the boundary mirrors the one
  inside), 8 -> 32 -> 32 -> 32 -> 4 channels.  Weights enter as BF16 (rounded
  from FP32 master copies), every sum is accumulated in FP32 (here: exactly
  in FP64, then rounded to FP32), the FP32 bias is added, and hidden layers
  store BF16(ReLU(.)).  The last layer's FP32 output y is not rounded.
* Guess: x1 + d + sigma * y (FP64): linear extrapolation of the previous
  increment plus a learned correction measured in units of the previous
  increment.  With a zero last layer the guess is linear extrapolation.
* Training target: t_c = (x0_c - x1_c - d_c) / sigma_c for the solution x0
  at step n.  Loss: the mean over samples s of w_s times the mean of
  (y - t)^2 over the masked pixels and the 4 channels of sample s (plus an
  optional penalty on differences of y - t between neighbouring pixels,
  loss_and_grad_output), with the
  sample weight w_s = 1 / (q_s + 1e-4), q_s the mean of t^2 over the whole
  grid and the 4 channels: every sample counts by its error relative to its
  own target, so the large targets of the first, fast steps of a run do not
  swamp the many small ones of its smooth later steps.
* Backward: the loss gradient is rounded to BF16, and so is every
  activation gradient after the ReLU mask; weight and bias gradients are FP32
  sums; the transpose of the reflective padding folds the padded border back
  onto rows/columns 1 and H-2 (W-2).
* Adam with bias correction, in FP32.
* Crops: training runs on crops of the feature grid; a crop is padded
  reflectively like the full grid, so outputs within 4 vertices (the
  receptive radius of four 3x3 layers) of a crop edge that lies inside the
  domain are masked out of the loss.
"""
from __future__ import annotations

import numpy as np

LAYERS = ((8, 32, True), (32, 32, True), (32, 32, True), (32, 4, False))  # (c_in, c_out, relu)
RADIUS = len(LAYERS)      # receptive radius in vertices
ADAM = dict(beta1=0.9, beta2=0.999, eps=1e-8)


# ---------------------------------------------------------------- BF16
def bf16(x) -> np.ndarray:
    """Round float32 values to bfloat16, round-to-nearest-even, returned as
    float32 holding the rounded value (finite inputs only)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return r.astype(np.uint32).view(np.float32).reshape(x.shape)


# ---------------------------------------------------------------- convolution
def pad_reflect(a: np.ndarray) -> np.ndarray:
    """[B, H, W, C] -> [B, H+2, W+2, C]; the border mirrors row/column 1 and
    H-2 / W-2 (needs H, W >= 2)."""
    return np.pad(a, ((0, 0), (1, 1), (1, 1), (0, 0)), mode="reflect")


def fold_reflect(g: np.ndarray) -> np.ndarray:
    """Adjoint of pad_reflect: [B, H+2, W+2, C] -> [B, H, W, C]."""
    t = np.array(g, dtype=np.float64, copy=True)
    H, W = t.shape[1] - 2, t.shape[2] - 2
    t[:, 2, :, :] += t[:, 0, :, :]          # padded row 0 is row 1
    t[:, H - 1, :, :] += t[:, H + 1, :, :]  # padded row H+1 is row H-2
    t = t[:, 1:H + 1]
    t[:, :, 2, :] += t[:, :, 0, :]
    t[:, :, W - 1, :] += t[:, :, W + 1, :]
    return t[:, :, 1:W + 1]


def conv(a: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """3x3 correlation with reflective padding, in FP64:
    out[b, i, j, o] = bias[o] + sum over dy, dx, c of
    pad(a)[b, i + dy, j + dx, c] * w[dy, dx, c, o]."""
    p = pad_reflect(np.asarray(a, dtype=np.float64))
    B, H, W = a.shape[0], a.shape[1], a.shape[2]
    out = np.zeros((B, H, W, w.shape[3]))
    for dy in range(3):
        for dx in range(3):
            out += p[:, dy:dy + H, dx:dx + W, :] @ np.asarray(w[dy, dx], dtype=np.float64)
    return out + np.asarray(b, dtype=np.float64)


def conv_grad_weights(a: np.ndarray, g: np.ndarray):
    """dL/dw[dy, dx, c, o] = sum over b, i, j of pad(a)[b, i+dy, j+dx, c] g[b, i, j, o];
    dL/dbias[o] = sum of g[..., o] (FP64)."""
    p = pad_reflect(np.asarray(a, dtype=np.float64))
    B, H, W = g.shape[0], g.shape[1], g.shape[2]
    g64 = np.asarray(g, dtype=np.float64).reshape(-1, g.shape[3])
    dw = np.zeros((3, 3, a.shape[3], g.shape[3]))
    for dy in range(3):
        for dx in range(3):
            dw[dy, dx] = p[:, dy:dy + H, dx:dx + W, :].reshape(-1, a.shape[3]).T @ g64
    return dw, g64.sum(axis=0)


def conv_grad_input(g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """dL/da for out = conv(a, w, .): scatter g through every tap into the padded
    grid, then fold the border back (FP64)."""
    B, H, W = g.shape[0], g.shape[1], g.shape[2]
    gp = np.zeros((B, H + 2, W + 2, w.shape[2]))
    g64 = np.asarray(g, dtype=np.float64)
    for dy in range(3):
        for dx in range(3):
            gp[:, dy:dy + H, dx:dx + W, :] += g64 @ np.asarray(w[dy, dx], dtype=np.float64).T
    return fold_reflect(gp)


# ---------------------------------------------------------------- network
def forward(params, feats: np.ndarray, quantize: bool = True):
    """Activations of every layer: acts[0] = the (BF16) input, acts[k] the BF16
    output of hidden layer k, and the FP32 output y of the last layer.
    quantize=False runs the same network in FP64 (for derivative checks)."""
    q = bf16 if quantize else (lambda v: np.asarray(v, dtype=np.float64))
    f32 = (lambda v: np.asarray(v, dtype=np.float32)) if quantize else (lambda v: v)
    acts = [q(feats)]
    a = acts[0]
    for (w, b), (_, _, relu) in zip(params, LAYERS):
        pre = f32(conv(a, q(w), np.asarray(b, dtype=np.float32 if quantize else np.float64)))
        if relu:
            a = q(np.maximum(pre, 0))
            acts.append(a)
        else:
            return acts, pre
    raise AssertionError("last layer must be linear")


WEIGHT_FLOOR = 1e-4


def loss_and_grad_output(y, t, mask, weights=None, smooth: float = 0.0, quantize: bool = True):
    """Loss = (1/B) sum over samples of w_s / (4 m_s) times the sum over the 4
    channels of [sum over masked pixels of e^2 + smooth * sum over the
    horizontal and vertical neighbour pairs with both pixels masked of
    (e_p - e_q)^2], e = y - t, m_s the masked pixels of sample s; and its
    gradient dL/dy (rounded to BF16 when quantize).  The pair term makes a
    rough error cost more than a smooth one of the same size.
    mask: [B, H, W] of 0/1; weights: [B] (None: all 1)."""
    B = y.shape[0]
    w = np.ones(B) if weights is None else np.asarray(weights, dtype=np.float64)
    m = np.asarray(mask, dtype=np.float64)[..., None]
    denom = 4.0 * m.reshape(B, -1).sum(axis=1) * B            # 4 m_s B per sample
    scale = (w / denom)[:, None, None, None]
    e = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    loss = float((scale * m * e * e).sum())
    g = 2.0 * m * e
    if smooth:
        ex = e[:, :, 1:] - e[:, :, :-1]
        mx = m[:, :, 1:] * m[:, :, :-1]
        ey = e[:, 1:] - e[:, :-1]
        my = m[:, 1:] * m[:, :-1]
        loss += smooth * float((scale * mx * ex * ex).sum() + (scale * my * ey * ey).sum())
        gx = 2.0 * smooth * mx * ex
        gyy = 2.0 * smooth * my * ey
        g[:, :, 1:] += gx
        g[:, :, :-1] -= gx
        g[:, 1:] += gyy
        g[:, :-1] -= gyy
    gy = w[:, None, None, None] * g / denom[:, None, None, None]
    return loss, (bf16(gy.astype(np.float32)) if quantize else gy)


def sample_weight(x2: np.ndarray, x1: np.ndarray, x0: np.ndarray, sigma: np.ndarray) -> float:
    """w = 1 / (mean over the grid and channels of t^2 + WEIGHT_FLOOR) (FP64)."""
    t = (x0 - x1 - (x1 - x2)) * _inv(sigma)[:, None, None]
    return 1.0 / (float(np.mean(np.mean(t * t, axis=(1, 2)))) + WEIGHT_FLOOR)


def backward(params, acts, gy, quantize: bool = True):
    """Gradients (dw, db) per layer, FP32 (FP64 when not quantize)."""
    q = bf16 if quantize else (lambda v: np.asarray(v, dtype=np.float64))
    f32 = (lambda v: np.asarray(v, dtype=np.float32)) if quantize else (lambda v: v)
    grads = [None] * len(params)
    g = gy
    for k in range(len(params) - 1, -1, -1):
        w = q(params[k][0])
        dw, db = conv_grad_weights(acts[k], g)
        grads[k] = (f32(dw), f32(db))
        if k == 0:
            break
        gin = conv_grad_input(g, w)
        g = q(f32(gin * (acts[k] > 0)))
    return grads


def adam(params, grads, m, v, t: int, lr: float, beta1=ADAM["beta1"], beta2=ADAM["beta2"],
         eps=ADAM["eps"]):
    """One Adam step (FP32) on every tensor; returns new params, m, v."""
    f = np.float32
    b1, b2, e, l = f(beta1), f(beta2), f(eps), f(lr)
    c1 = f(1.0 - beta1 ** t)     # bias corrections: FP64, rounded once to FP32
    c2 = f(1.0 - beta2 ** t)
    out_p, out_m, out_v = [], [], []
    for P, G, M, V in zip(params, grads, m, v):
        np_, nm, nv = [], [], []
        for p_, g_, m_, v_ in zip(P, G, M, V):
            g32 = np.asarray(g_, dtype=f)
            m1 = b1 * m_ + (f(1) - b1) * g32
            v1 = b2 * v_ + (f(1) - b2) * (g32 * g32)
            step = l * (m1 / c1) / (np.sqrt(v1 / c2) + e)
            np_.append((p_ - step).astype(f))
            nm.append(m1.astype(f))
            nv.append(v1.astype(f))
        out_p.append(tuple(np_))
        out_m.append(tuple(nm))
        out_v.append(tuple(nv))
    return out_p, out_m, out_v


def zeros_like_params(params):
    return [tuple(np.zeros_like(np.asarray(x, dtype=np.float32)) for x in layer) for layer in params]


# ---------------------------------------------------------------- features, guess, targets
def _rms(a):
    return np.sqrt(np.mean(a * a, axis=(1, 2)))


def _inv(s):
    return np.where(s > 0, 1.0 / np.where(s > 0, s, 1.0), 0.0)


def features(x2: np.ndarray, x1: np.ndarray, quantize: bool = True):
    """x2, x1: [4, H, W] FP64 states at steps n-2 and n-1.  Returns the [H, W, 8]
    feature grid (BF16 values in float32 when quantize) and sigma [4]."""
    d = x1 - x2
    sigma = _rms(d)
    xc = x1 - x1.mean(axis=(1, 2), keepdims=True)
    tau = _rms(xc)
    f = np.concatenate([d * _inv(sigma)[:, None, None], xc * _inv(tau)[:, None, None]])
    f = np.moveaxis(f, 0, -1)
    return (bf16(f.astype(np.float32)) if quantize else f), sigma


def target(x2: np.ndarray, x1: np.ndarray, x0: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    """[H, W, 4] FP32 training target for the solution x0 at step n."""
    t = (x0 - x1 - (x1 - x2)) * _inv(sigma)[:, None, None]
    return np.moveaxis(t, 0, -1).astype(np.float32)


def guess(x2: np.ndarray, x1: np.ndarray, y: np.ndarray, sigma: np.ndarray) -> np.ndarray:
    """[4, H, W] FP64 guess x1 + d + sigma * y from the [H, W, 4] output y."""
    return x1 + (x1 - x2) + sigma[:, None, None] * np.moveaxis(np.asarray(y, dtype=np.float64), -1, 0)


def crop_mask(H: int, W: int, oy: int, ox: int, h: int, w: int) -> np.ndarray:
    """[h, w] 0/1: 0 within RADIUS of a crop edge that lies inside the domain."""
    m = np.ones((h, w))
    if oy > 0:
        m[:RADIUS, :] = 0
    if oy + h < H:
        m[h - RADIUS:, :] = 0
    if ox > 0:
        m[:, :RADIUS] = 0
    if ox + w < W:
        m[:, w - RADIUS:] = 0
    return m


def fields_grid(phi_p, phi_n, mu_p, mu_n, H: int, W: int) -> np.ndarray:
    """[4, H, W] from four vertex vectors of length H * W (vertex = row * W + col)."""
    return np.stack([np.asarray(a, dtype=np.float64).reshape(H, W) for a in (phi_p, phi_n, mu_p, mu_n)])
