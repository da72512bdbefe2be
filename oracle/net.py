"""Oracle for the learned candidate classifier (test infrastructure only).

The paper screens its Stage I candidates with automated cuts and visual inspection (Stage II,
Sec. 2.4: extended, horizon-hugging and image-wide structures are rejected).  The classifier
stands in for that screen; the paper gives no network, so everything below is this project's
reading, stated once here and followed by the GPU path:

* Candidate stamp: the detector's SNR cube around a candidate (c, y, x), 33 channels
  (c - 16 .. c + 16) by 9 x 9 pixels (y - 4 .. y + 4, x - 4 .. x + 4), zero outside the cube;
  layout [33][9][9], channel-major.
* Network: three 3 x 3 convolutions with zero padding 1 (33 -> 32 -> 64 -> 32 channels, the
  spectral channels of the stamp are the input channels), each followed by ReLU; global
  average pool over the 9 x 9 positions; one linear unit; the logit z scores "sky-localised
  narrowband tone" (label 1) against RFI, artefacts and noise (label 0).
* Convolution as cross-correlation:
      Z[o][y][x] = b[o] + sum_{i, dy, dx} W[o][i][dy][dx] X[i][y + dy - 1][x + dx - 1].
* Loss: binary cross-entropy on the logit, averaged over the batch:
      L = (1/B) sum_b [ log(1 + e^{z_b}) - y_b z_b ],  dL/dz_b = (sigmoid(z_b) - y_b) / B.
* Optimizer: Adam (Kingma & Ba, 2015) on FP32 master weights:
      m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
      theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Flat parameter vector (float, 46,529 entries), in this order:
  W1[32][33][3][3], b1[32], W2[64][32][3][3], b2[64], W3[32][64][3][3], b3[32], w4[32], b4[1].

Everything here is float64 numpy; np.einsum over the nine shifted copies of the padded input
is the only library primitive.
"""
from __future__ import annotations

import numpy as np

STAMP_C = 33
STAMP_P = 9
HALF_C = STAMP_C // 2
HALF_P = STAMP_P // 2
LAYERS = [(33, 32), (32, 64), (64, 32)]  # (in, out) channels of the three convolutions
SHAPES = [("W1", (32, 33, 3, 3)), ("b1", (32,)), ("W2", (64, 32, 3, 3)), ("b2", (64,)),
          ("W3", (32, 64, 3, 3)), ("b3", (32,)), ("w4", (32,)), ("b4", (1,))]
N_PARAM = int(sum(np.prod(s) for _, s in SHAPES))


def unpack(theta: np.ndarray) -> dict:
    """Flat vector -> named float64 arrays (copies)."""
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp).copy()
        o += n
    assert o == N_PARAM == theta.size
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def stamps(cube: np.ndarray, cands) -> np.ndarray:
    """Stamps [n][33][9][9] of cube [C][N][N] around candidates (c, y, x), zero outside."""
    C, N, _ = cube.shape
    out = np.zeros((len(cands), STAMP_C, STAMP_P, STAMP_P), dtype=np.float64)
    for k, (c, y, x) in enumerate(cands):
        for dc in range(STAMP_C):
            cc = c + dc - HALF_C
            if not 0 <= cc < C:
                continue
            for dy in range(STAMP_P):
                yy = y + dy - HALF_P
                if not 0 <= yy < N:
                    continue
                for dx in range(STAMP_P):
                    xx = x + dx - HALF_P
                    if 0 <= xx < N:
                        out[k, dc, dy, dx] = cube[cc, yy, xx]
    return out


def _shifts(X: np.ndarray) -> np.ndarray:
    """The nine zero-padded shifts of X [B][I][H][W]: S[dy][dx][b][i][y][x] = X[b][i][y+dy-1][x+dx-1]."""
    B, I, H, W = X.shape
    P = np.zeros((B, I, H + 2, W + 2), dtype=np.float64)
    P[:, :, 1:H + 1, 1:W + 1] = X
    return np.stack([np.stack([P[:, :, dy:dy + H, dx:dx + W] for dx in range(3)]) for dy in range(3)])


def conv3x3(X: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Z[b][o][y][x] = bias[o] + sum_{i,dy,dx} W[o][i][dy][dx] X[b][i][y+dy-1][x+dx-1]."""
    return np.einsum("oiuv,uvbiyx->boyx", W, _shifts(X)) + b[None, :, None, None]


def conv3x3_backward(X: np.ndarray, W: np.ndarray, dZ: np.ndarray):
    """Gradients of sum(dZ * conv3x3(X, W, b)) with respect to X, W and b."""
    S = _shifts(X)
    dW = np.einsum("boyx,uvbiyx->oiuv", dZ, S)
    db = dZ.sum(axis=(0, 2, 3))
    # X[i][y'][x'] meets Z[o][y][x] through tap (dy, dx) when y' = y + dy - 1, x' = x + dx - 1
    B, I, H, Wd = X.shape
    dP = np.zeros((B, I, H + 2, Wd + 2), dtype=np.float64)
    for dy in range(3):
        for dx in range(3):
            dP[:, :, dy:dy + H, dx:dx + Wd] += np.einsum("oi,boyx->biyx", W[:, :, dy, dx], dZ)
    return dP[:, :, 1:H + 1, 1:Wd + 1], dW, db


def forward(theta: np.ndarray, X: np.ndarray):
    """Logits z [B] of stamps X [B][33][9][9], and the cache the backward pass needs."""
    p = unpack(theta)
    acts = [np.asarray(X, dtype=np.float64)]
    zs = []
    for l in range(3):
        Z = conv3x3(acts[-1], p[f"W{l + 1}"], p[f"b{l + 1}"])
        zs.append(Z)
        acts.append(np.maximum(Z, 0.0))
    feat = acts[-1].mean(axis=(2, 3))                     # global average pool [B][32]
    z = feat @ p["w4"] + p["b4"][0]
    return z, (p, acts, zs, feat)


def bce(z: np.ndarray, y: np.ndarray) -> float:
    """Mean binary cross-entropy on logits, log(1 + e^z) - y z, evaluated stably."""
    z = np.asarray(z, dtype=np.float64)
    return float(np.mean(np.logaddexp(0.0, z) - y * z))


def sigmoid(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def loss_and_grad(theta: np.ndarray, X: np.ndarray, y: np.ndarray):
    """Mean BCE over the batch and its gradient with respect to the flat parameter vector."""
    y = np.asarray(y, dtype=np.float64)
    z, (p, acts, zs, feat) = forward(theta, X)
    B = z.size
    dz = (sigmoid(z) - y) / B
    g = {"w4": feat.T @ dz, "b4": np.array([dz.sum()])}
    H = acts[-1].shape[2] * acts[-1].shape[3]
    dA = (dz[:, None] * p["w4"][None, :])[:, :, None, None] / H * np.ones_like(acts[-1])
    for l in (2, 1, 0):
        dZ = dA * (zs[l] > 0)
        dX, dW, db = conv3x3_backward(acts[l], p[f"W{l + 1}"], dZ)
        g[f"W{l + 1}"], g[f"b{l + 1}"] = dW, db
        dA = dX
    return bce(z, y), pack(g)


def adam(theta, m, v, g, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (t counts from 1); returns the new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
