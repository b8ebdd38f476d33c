"""Learned (k, p, q) predictor: the small MLP and its pilot-sketch features,
FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper chooses R_SVD and p by hand (section "Randomized matrix
decompositions"; R% swept in the results). This addition predicts them per
channel from a cheap pilot sketch, so most channels need no adaptive growth:

  features  Y0 = V P0 with a 32-column projection P0 (operands rounded to
            FP32, as the pilot runs on FP32 matrix cores); s_i = singular
            values of Y0; f_i = max(log10(s_i / s_1), -16), i = 1..16
  model     h1 = relu(W1 f + b1)      W1: 64 x 16
            h2 = relu(W2 h1 + b2)     W2: 64 x 64
            y  = W3 h2 + b3           W3: 3 x 64      (5443 parameters)
            y estimates the standardized targets (log10 k, p, q)
  loss      mean over the batch and the 3 outputs of (y - t)^2
  optimizer Adam (Kingma and Ba 2015): m <- b1 m + (1 - b1) g,
            v <- b2 v + (1 - b2) g^2, w <- w - lr mhat / (sqrt(vhat) + eps),
            mhat = m / (1 - b1^t), vhat = v / (1 - b2^t)
  init      He (Kaiming) normal: W ~ N(0, 2 / fan_in), biases 0; the normal
            draws are the Philox4x64-10 / Box-Muller stream keyed by
            (seed, layer index), entry (i, j) of layer L at row i, column j
            of an out x in matrix

Parameter layout (one flat FP32 vector on the device, the same order here):
W1 (64 x 16, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (3 x 64), b3 (3).

Sizing (the same rules as the device): targets() standardizes integer labels
(log10 k, p, q) by their column means and population deviations; decode()
turns a network output back into (k, p, q) with a 5 % rank margin and the
grids p in {8, 16, 32, 48, 64, 96, 128, 160, 192, 256, 320, 384, 448, 512},
q in 0..4; size_label() picks a label
from a spectrum the method computed: the cheapest grid point whose kept
values are converged, (s_{k+p}/s_k)^(4q+2) <= 1e-8, by the cost of the
products with A, the panel QRs and the small SVD (seconds, fitted to the
library's measured times).

Pins (tests/test_oracle_mlp.py): hand-worked standardization, decoding and
labels; fourth-order finite-difference gradients
of the loss, Adam against its closed form for the first steps, the He
moments, the feature map on matrices with known spectra (slope of a
10^(-i/4) spectrum, the rounding floor of a rank-1 matrix, exact invariance
under power-of-two scaling), and learning of a known linear relation.
"""

import math

import numpy as np

from .philox import gaussian_omega

N_IN, N_HID, N_OUT = 16, 64, 3
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 5443
PILOT_COLS = 32
FEATURE_FLOOR = -16.0


def unpack(theta):
    """Flat parameter vector -> dict of arrays (views)."""
    out, at = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[at:at + size].reshape(shape)
        at += size
    return out


def he_init(seed):
    """He-normal weights from the Philox/Box-Muller stream, zero biases."""
    theta = np.zeros(N_PARAMS)
    p = unpack(theta)
    for layer, name in enumerate(("W1", "W2", "W3")):
        rows, cols = p[name].shape
        # gaussian_omega(n, l, seed, channel) gives entry (i, j) at counter (i, j/4)
        z = gaussian_omega(rows, cols, seed, layer)
        p[name][...] = z * math.sqrt(2.0 / cols)
    return theta


def forward(theta, X):
    """Outputs (B x 3) and the activations needed by backward."""
    p = unpack(theta)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (X, z1, h1, z2, h2)


def loss(theta, X, T):
    y, _ = forward(theta, X)
    return float(np.mean((y - T) ** 2))


def grad(theta, X, T):
    """Analytic gradient of loss() (backpropagation); returns (loss, g)."""
    p = unpack(theta)
    y, (X, z1, h1, z2, h2) = forward(theta, X)
    B = X.shape[0]
    dy = 2.0 * (y - T) / (B * N_OUT)
    g = np.zeros_like(theta)
    gp = unpack(g)
    gp["W3"][...] = dy.T @ h2
    gp["b3"][...] = dy.sum(axis=0)
    dh2 = dy @ p["W3"]
    dz2 = dh2 * (z2 > 0.0)
    gp["W2"][...] = dz2.T @ h1
    gp["b2"][...] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0.0)
    gp["W1"][...] = dz1.T @ X
    gp["b1"][...] = dz1.sum(axis=0)
    return float(np.mean((y - T) ** 2)), g


ADAM = dict(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8)


def adam_step(theta, m, v, g, t, lr=ADAM["lr"], beta1=ADAM["beta1"], beta2=ADAM["beta2"],
              eps=ADAM["eps"]):
    """One Adam update at step t >= 1 (new theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(theta, X, T, epochs, batch=128, lr=ADAM["lr"]):
    """Plain minibatch Adam over the rows of X in order (no shuffling)."""
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    t = 0
    hist = []
    for _ in range(epochs):
        for b0 in range(0, X.shape[0], batch):
            t += 1
            L, g = grad(theta, X[b0:b0 + batch], T[b0:b0 + batch])
            theta, m, v = adam_step(theta, m, v, g, t, lr=lr)
            hist.append(L)
    return theta, hist


def pilot_features(A, seed, channel=0):
    """f_i = max(log10(s_i(Y0) / s_1(Y0)), -16), i = 1..16, Y0 = fp32(A) fp32(P0)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    P0 = gaussian_omega(n, PILOT_COLS, seed, channel)
    A32 = A.astype(np.float32).astype(np.float64)
    P32 = P0.astype(np.float32).astype(np.float64)
    Y0 = A32 @ P32
    s = np.linalg.svd(Y0, compute_uv=False)
    f = np.full(N_IN, FEATURE_FLOOR)
    if s[0] > 0:
        r = s[:N_IN] / s[0]
        with np.errstate(divide="ignore"):
            f[: len(r)] = np.maximum(np.log10(r), FEATURE_FLOOR)
    return f


# ---- sizing from the network and labels from computed spectra ---------------
P_GRID = (8, 16, 32, 48, 64, 96, 128, 160, 192, 256, 320, 384, 448, 512)
Q_MAX = 4
RANK_MARGIN = 1.05
# cost of a decomposition of width l, in seconds fitted to the library's
# measured times: 2q + 2 products with A at 60 TFLOP/s and as many panel QRs
# (2q + 1 in the power iteration, one of the projection) at
# QR_SECONDS (l / 272)^1.6 each, plus the small SVD at SVD_SECONDS (l / 272)^1.6
PRODUCT_FLOPS = 60e12
QR_SECONDS = 0.44e-3
SVD_SECONDS = 3.2e-3


def targets(labels):
    """Raw targets (log10 k, p, q) of integer labels, their column means and
    population standard deviations (0 -> 1), and the standardized targets."""
    L = np.asarray(labels, dtype=np.float64).reshape(-1, 3)
    raw = np.stack([np.log10(np.maximum(L[:, 0], 1.0)), L[:, 1], L[:, 2]], axis=1)
    mean = raw.mean(axis=0)
    sd = raw.std(axis=0)
    sd[sd == 0] = 1.0
    return (raw - mean) / sd, mean, sd


def decode(y, mean, sd, n_cap):
    """Network output y (3 values, standardized) -> (k, p, q): k with a 5 %
    margin rounded up into 1..n_cap, p rounded up to the grid (512 beyond it),
    q rounded to nearest into 0..4."""
    raw = [float(y[i]) * float(sd[i]) + float(mean[i]) for i in range(3)]
    kk = math.ceil(RANK_MARGIN * 10.0 ** raw[0]) if raw[0] < 300 else math.inf
    k = int(min(max(kk, 1), n_cap))
    p = next((g for g in P_GRID if g >= raw[1]), P_GRID[-1])
    q = int(min(max(math.floor(raw[2] + 0.5), 0), Q_MAX))
    return k, p, q


def size_label(s, k, n, l_min=0):
    """Cheapest (p, q) on the grid whose l = k + p reaches n, or whose l is at
    least l_min (the width at which the labelling run's posterior estimate
    passed) and whose kept values are converged on the computed spectrum s
    (decreasing): (s[k+p-1] / s[k-1])^(4q+2) <= 1e-8, the last computed value
    standing in beyond len(s) (the ratio only falls further). Returns
    (k, p, q), with p = q = -1 when no grid point qualifies."""
    best = None
    for q in range(Q_MAX + 1):
        for p in P_GRID:
            if k + p < n:
                if k + p < l_min:
                    continue
                j = min(k + p, len(s))
                if j <= k:
                    continue
                r = s[j - 1] / s[k - 1] if s[k - 1] > 0 else 0.0
                if not r ** (4 * q + 2) <= 1e-8:
                    continue
            L = min(k + p, n)
            w = (L / 272.0) ** 1.6
            cost = (2 * q + 2) * (2.0 * n * n * L / PRODUCT_FLOPS + QR_SECONDS * w) + SVD_SECONDS * w
            if best is None or cost < best[0]:
                best = (cost, p, q)
    return (k, best[1], best[2]) if best else (k, -1, -1)
