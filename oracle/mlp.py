"""FP64 CPU oracle of the learned warm start -- TEST INFRASTRUCTURE.

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may use
this module; it shares no code with the HIP path.

The warm start is not part of the paper: Algorithm 1 starts every message at
zero (step 1).  Here a small per-node network proposes initial messages for
the structured-grid operators of section IX instead; the solver's own
iteration then proceeds unchanged, so the fixed point, and the answer
x = A^{-1} b, are the paper's whatever the network outputs.

Network (plain numpy, float64):
    u  in R^8   node features
    h1 = relu(W1 u + b1)          W1: 64 x 8
    h2 = relu(W2 h1 + b2)         W2: 64 x 64
    o  = W3 h2 + b3               W3: 12 x 64
Flat parameter order: W1 (row-major), b1, W2, b2, W3, b3 (5516 values).
Loss of a batch: sum over samples s and unmasked outputs j of
(o_sj - t_sj)^2, divided by 2 x (number of unmasked outputs).

Features of grid node i (directions +x, -x, +y, -y, +z, -z; a_d = A_{i,j(d)},
0 where the neighbour is outside the grid):
    u = (log A_ii, a_1 / A_ii, ..., a_6 / A_ii, b_i / A_ii)
Targets (the converged messages i -> j(d) in the information form of
section III-C, h = P mu): t_{2d} = P_d / A_ii, t_{2d+1} = h_d / A_ii, masked
where a_d = 0.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 8, 64, 12
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    """Flat parameter vector -> dict of arrays (views)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as
    float64.  bfloat16 keeps the top 16 bits of the float32 pattern."""
    f = np.asarray(x, dtype=np.float32).copy()
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta, U):
    """Outputs (S x 12) and the activations needed by backward."""
    p = unpack(theta)
    U = np.asarray(U, dtype=np.float64)
    z1 = U @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    o = h2 @ p["W3"].T + p["b3"]
    return o, (U, z1, h1, z2, h2)


def loss(theta, U, T, M):
    """Masked mean squared error / 2 (M: 1 where the output counts)."""
    o, _ = forward(theta, U)
    n = float(np.sum(M))
    return 0.5 * float(np.sum(M * (o - T) ** 2)) / max(n, 1.0)


def grad(theta, U, T, M):
    """(loss, flat gradient) by the chain rule through the three layers."""
    p = unpack(theta)
    o, (U, z1, h1, z2, h2) = forward(theta, U)
    n = max(float(np.sum(M)), 1.0)
    d_o = M * (o - T) / n                      # dL/do
    g = {"W3": d_o.T @ h2, "b3": d_o.sum(axis=0)}
    d_h2 = d_o @ p["W3"]
    d_z2 = d_h2 * (z2 > 0)
    g["W2"] = d_z2.T @ h1
    g["b2"] = d_z2.sum(axis=0)
    d_h1 = d_z2 @ p["W2"]
    d_z1 = d_h1 * (z1 > 0)
    g["W1"] = d_z1.T @ U
    g["b1"] = d_z1.sum(axis=0)
    L = 0.5 * float(np.sum(M * (o - T) ** 2)) / n
    return L, pack(g)


def adam_step(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) of the FP32 master parameters; step
    counts from 1.  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# grid features and targets
# ---------------------------------------------------------------------------
def _neighbours(nx, ny, nz, batch):
    """(node count, list of 6 (neighbour index or -1) arrays) in the order
    +x, -x, +y, -y, +z, -z, natural ordering i = x + nx (y + ny z) per grid."""
    n = nx * ny * nz
    i = np.arange(n * batch)
    loc = i % n
    x = loc % nx
    y = (loc // nx) % ny
    z = loc // (nx * ny)
    nb = [np.where(x + 1 < nx, i + 1, -1), np.where(x > 0, i - 1, -1),
          np.where(y + 1 < ny, i + nx, -1), np.where(y > 0, i - nx, -1),
          np.where(z + 1 < nz, i + nx * ny, -1), np.where(z > 0, i - nx * ny, -1)]
    return n * batch, nb


def grid_couplings(nx, ny, nz, batch, coef):
    """(A_ii per node, 6 x N couplings a_d, 0 where no neighbour) from the
    coefficient dict of workloads.grid_stack (per-node diag and +x/+y/+z face
    couplings, or constants dval/off)."""
    N, nb = _neighbours(nx, ny, nz, batch)
    if coef.get("diag") is not None:
        diag = np.asarray(coef["diag"], dtype=np.float64)
        cx, cy, cz = (np.asarray(coef[k], dtype=np.float64) for k in ("cx", "cy", "cz"))
    else:
        diag = np.full(N, float(coef["dval"]))
        cx = cy = cz = np.full(N, float(coef["off"]))
    a = np.zeros((6, N))
    for d, (c, step) in enumerate(((cx, 1), (cy, nx), (cz, nx * ny))):
        plus, minus = nb[2 * d], nb[2 * d + 1]
        ok = plus >= 0
        a[2 * d, ok] = c[ok]                      # A_{i, i+step} stored at i
        ok = minus >= 0
        a[2 * d + 1, ok] = c[minus[ok]]           # A_{i, i-step} stored at i-step
    return diag, a


def grid_features(nx, ny, nz, batch, coef, b):
    diag, a = grid_couplings(nx, ny, nz, batch, coef)
    b = np.asarray(b, dtype=np.float64)
    U = np.empty((diag.size, N_IN))
    U[:, 0] = np.log(diag)
    U[:, 1:7] = (a / diag).T
    U[:, 7] = b / diag
    return U


def grid_targets(nx, ny, nz, batch, coef, P, h):
    """Targets and mask from messages P, h laid out [6][N] (message from node
    i toward direction d at [d][i])."""
    diag, a = grid_couplings(nx, ny, nz, batch, coef)
    P = np.asarray(P, dtype=np.float64).reshape(6, -1)
    h = np.asarray(h, dtype=np.float64).reshape(6, -1)
    T = np.zeros((diag.size, N_OUT))
    M = np.zeros((diag.size, N_OUT))
    for d in range(6):
        on = a[d] != 0
        T[:, 2 * d] = np.where(on, P[d] / diag, 0.0)
        T[:, 2 * d + 1] = np.where(on, h[d] / diag, 0.0)
        M[:, 2 * d] = on
        M[:, 2 * d + 1] = on
    return T, M
