"""Learned per-patch surrogate: plain FP64 reference (test infrastructure only).

Per coarse element (patch) K a multilayer perceptron maps the patch's local
random variables (the xi_j whose mode touches K, Sec. 3 eq. MsFEB2; zero
padded to k_in inputs) to the 10 unique entries of the upscaled stiffness,
standardised per entry with the training mean and standard deviation:

    Z1 = X W1 + b1, H1 = gelu(Z1), Z2 = H1 W2 + b2, H2 = gelu(Z2),
    Z3 = H2 W3 + b3, H3 = gelu(Z3), Y = H3 W4 + b4,

with gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2 and Y holding two
independent output heads of 10 entries each.  Loss: mean squared error of
both heads against the standardised targets,
    L = (1 / (B * 20)) sum_b sum_o (Y_bo - T_b,(o mod 10))^2.
Gradients by hand-written reverse mode; Adam (Kingma & Ba) for the update.

Gate (a reading of the residual/uncertainty gate): for a prediction with heads
S_A, S_B (de-standardised, unpacked to 4x4), S = (S_A + S_B) / 2,
    residual    = max_l |sum_l' S_ll'| / max |S|   (S 1 = 0 for every exact S)
    uncertainty = max |S_A - S_B| / max |S|
and the pair is accepted when max(residual, uncertainty) <= tau and every
local variable lies inside the training box; accepted predictions are
projected onto the zero-row-sum matrices, S <- P S P with P = I - 1 1^T / 4.

Parameter packing (float, per patch): W1 [k_in][64], b1 [64], W2 [64][64],
b2 [64], W3 [64][64], b3 [64], W4 [64][20], b4 [20] (row-major, in this order).
"""
from __future__ import annotations

import math

import numpy as np

WIDTH = 64
NOUT = 10
HEADS = 2


def layer_shapes(kin: int):
    return [(kin, WIDTH), (WIDTH,), (WIDTH, WIDTH), (WIDTH,), (WIDTH, WIDTH), (WIDTH,),
            (WIDTH, HEADS * NOUT), (HEADS * NOUT,)]


def nparams(kin: int) -> int:
    return sum(int(np.prod(s)) for s in layer_shapes(kin))


def unpack_params(flat: np.ndarray, kin: int) -> list[np.ndarray]:
    out, o = [], 0
    for s in layer_shapes(kin):
        n = int(np.prod(s))
        out.append(np.asarray(flat[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def pack_params(ps: list[np.ndarray]) -> np.ndarray:
    return np.concatenate([p.ravel() for p in ps])


def _erf(z):
    return np.vectorize(math.erf)(z)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    Phi = 0.5 * (1.0 + _erf(z / math.sqrt(2.0)))
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return Phi + z * phi


def forward(flat: np.ndarray, X: np.ndarray, kin: int):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack_params(flat, kin)
    Z1 = X @ W1 + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2 + b2
    H2 = gelu(Z2)
    Z3 = H2 @ W3 + b3
    H3 = gelu(Z3)
    Y = H3 @ W4 + b4
    return Y, (X, Z1, H1, Z2, H2, Z3, H3)


def loss(Y: np.ndarray, T: np.ndarray) -> float:
    T2 = np.concatenate([T, T], axis=1)
    return float(np.mean((Y - T2) ** 2))


def grad(flat: np.ndarray, X: np.ndarray, T: np.ndarray, kin: int):
    """(loss, flat gradient) by reverse mode."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack_params(flat, kin)
    Y, (X, Z1, H1, Z2, H2, Z3, H3) = forward(flat, X, kin)
    B = X.shape[0]
    T2 = np.concatenate([T, T], axis=1)
    dY = 2.0 * (Y - T2) / (B * HEADS * NOUT)
    gW4 = H3.T @ dY
    gb4 = dY.sum(0)
    dZ3 = (dY @ W4.T) * gelu_grad(Z3)
    gW3 = H2.T @ dZ3
    gb3 = dZ3.sum(0)
    dZ2 = (dZ3 @ W3.T) * gelu_grad(Z2)
    gW2 = H1.T @ dZ2
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2.T) * gelu_grad(Z1)
    gW1 = X.T @ dZ1
    gb1 = dZ1.sum(0)
    return loss(Y, T), pack_params([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4])


def adam_step(flat, g, m1, m2, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (flat, m1, m2)."""
    m1 = beta1 * m1 + (1 - beta1) * g
    m2 = beta2 * m2 + (1 - beta2) * g * g
    mh = m1 / (1 - beta1**t)
    vh = m2 / (1 - beta2**t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m1, m2


def standardize(S_train: np.ndarray):
    """Per-entry mean and std of training targets [N][10]; std floored at
    1e-12 * max|mean| so that constant entries stay finite."""
    mu = S_train.mean(0)
    sd = S_train.std(0)
    floor = 1e-12 * max(1.0, float(np.abs(mu).max()))
    return mu, np.maximum(sd, floor)


PACK = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]


def _unpack4(s10):
    S = np.zeros(s10.shape[:-1] + (4, 4))
    for q, (i, j) in enumerate(PACK):
        S[..., i, j] = s10[..., q]
        S[..., j, i] = s10[..., q]
    return S


def gate(Y: np.ndarray, mu: np.ndarray, sd: np.ndarray, X: np.ndarray, nlocal: int, tau: float, box: float = 1.0,
         scale: np.ndarray | None = None):
    """Y [B][20] raw network outputs -> (accepted mask [B], S [B][10] packed,
    residual [B], uncertainty [B]).  scale [B] (optional): the network
    predicts S / scale (a per-pair output scale), so both heads are multiplied
    by it after de-standardisation; the two signals are ratios of entries of
    S and do not change with it."""
    osc = np.ones(len(Y)) if scale is None else np.asarray(scale, dtype=np.float64)
    SA = osc[:, None] * (mu + sd * Y[:, :NOUT])
    SB = osc[:, None] * (mu + sd * Y[:, NOUT:])
    S = 0.5 * (SA + SB)
    S4 = _unpack4(S)
    scale = np.abs(S).max(-1)
    resid = np.abs(S4.sum(-1)).max(-1) / scale
    unc = np.abs(SA - SB).max(-1) / scale
    inbox = np.all(np.abs(X[:, :nlocal]) <= box, axis=1)
    ok = (np.maximum(resid, unc) <= tau) & inbox
    P = np.eye(4) - np.ones((4, 4)) / 4.0
    Sp = P @ S4 @ P
    packed = np.stack([Sp[:, i, j] for (i, j) in PACK], axis=-1)
    return ok, packed, resid, unc


# --- channels-and-inclusions medium ------------------------------------------
# A reading for this medium (its conductivities theta_j = 10^(d sigma(xi_j)),
# sigma the logistic function, span d decades): the network input of a local
# feature is u_j = 2 sigma(xi_j) - 1, the covered fraction of the decades
# mapped to [-1, 1], and the predicted quantity is S_K divided by the mean of
# the coefficient over the fine elements that touch the boundary of K (with
# linear boundary conditions those elements carry the prescribed gradient, so
# max |S_K| follows this mean over the decades; the mean over all of K, or
# 1 + sum_j theta_j, do not).


def local_features(fmap: np.ndarray, ncx: int, ncy: int, m: int) -> list[list[int]]:
    """Sorted distinct feature indices covering a fine element of each coarse
    element K = ky*ncx + kx (fmap [ncy*m][ncx*m], -1 = background)."""
    out = []
    for ky in range(ncy):
        for kx in range(ncx):
            blk = fmap[ky * m:(ky + 1) * m, kx * m:(kx + 1) * m]
            out.append(sorted({int(v) for v in blk.ravel() if v >= 0}))
    return out


def features_input(xi: np.ndarray) -> np.ndarray:
    """u = 2 / (1 + exp(-xi)) - 1."""
    return 2.0 / (1.0 + np.exp(-xi)) - 1.0


def ring_mean(a_blk: np.ndarray) -> float:
    """Mean of an m x m coefficient block over its boundary ring of fine
    elements (each element once)."""
    m = a_blk.shape[0]
    ring = np.zeros((m, m), dtype=bool)
    ring[0, :] = ring[-1, :] = ring[:, 0] = ring[:, -1] = True
    return float(a_blk[ring].mean())
