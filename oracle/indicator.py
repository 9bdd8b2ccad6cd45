"""Oracle: per-cell smoothness features and the blending-weight MLP (FP64).

Test infrastructure only.  The learned indicator is not in the paper: it maps
normalised DOLINC quantities of a cell to a weight theta in [0, 1] that blends
the high-order face state with the Van Leer limited one.

Features (24 per cell): four channels q in {rho, p, rho E, |rho u|}, six
statistics each, over the faces of the cell taken in the frame where the
cell is upwind (phi_0 = q of the cell, phi_1 = q of the neighbour,
d0 = centre distance pointing away from the cell):
    Delta = phi_1 - phi_0,  g0 = 2 d0 . grad q  (the DOLINC differential,
    Sec. 2.3),  s = g0 - Delta  (the upwind difference g (phi_0 - phi_-1)),
    beta = |s - Delta| / (|s| + |Delta| + eps),  scale = |q| + mean |Delta|.
    f1 = max |g0| / scale      f2 = max |Delta| / scale
    f3 = max beta              f4 = mean beta
    f5 = min clip(s Delta / (Delta^2 + eps^2), -2, 2)
    f6 = max |s - Delta| / scale
  each clipped to [-8, 8].  grad p and grad |rho u| come from the gradients
  of the conserved variables by the chain rule.
Network: 24 -> 64 (tanh) -> 64 (tanh) -> 1 (sigmoid).  Loss: binary cross
entropy on soft labels, averaged over the batch.  Optimiser: Adam.
With ``bf16=True`` the forward and backward passes round X, W1, W2, H1 and
the back-propagated deltas to bfloat16 (round to nearest even) at the points
where the GPU kernels feed matrix-core operands; everything else is exact.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 24, 64
N_PARAMS = N_H * N_IN + N_H + N_H * N_H + N_H + N_H + 1


def bf16_round(x):
    """Round float values to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ------------------------------------------------------------------ features
def channels(U, G1, gamma):
    """Cell values and gradients of rho, p, rho E, |rho u| -> ([nc,4], [nc,4,d])."""
    rho = U[:, 0]
    m = U[:, 1:4]
    E = U[:, 4]
    u = m / rho[:, None]
    ke = 0.5 * np.sum(m * u, 1)
    p = (gamma - 1.0) * (E - ke)
    mag = np.linalg.norm(m, axis=1)
    g_rho, g_m, g_E = G1[:, 0], G1[:, 1:4], G1[:, 4]
    u_dot_gm = np.einsum("ca,cad->cd", u, g_m)
    g_p = (gamma - 1.0) * (g_E - u_dot_gm + 0.5 * np.sum(u * u, 1)[:, None] * g_rho)
    safe = np.where(mag > 1e-30, mag, 1.0)
    g_mag = np.where((mag > 1e-30)[:, None], np.einsum("ca,cad->cd", m / safe[:, None], g_m), 0.0)
    q = np.stack([rho, p, E, mag], 1)
    gq = np.stack([g_rho, g_p, g_E, g_mag], 1)
    return q, gq


def features(mesh, geo, U, G1, gamma=1.4):
    """[nc, 24] features of every cell (see module docstring)."""
    q, gq = channels(U, G1, gamma)
    nc = mesh.n_cells
    P, N = mesh.owner, mesh.neighbour
    out = np.zeros((nc, 24))
    for k in range(4):
        stats = {n: None for n in ("g0", "dl", "beta", "r", "sd")}
        acc_max = [np.zeros(nc) for _ in range(5)]
        acc_min = np.full(nc, np.inf)
        sum_beta = np.zeros(nc)
        sum_dl = np.zeros(nc)
        cnt = np.zeros(nc)
        for side in (0, 1):
            c = P if side == 0 else N
            o = N if side == 0 else P
            d0 = geo.d if side == 0 else -geo.d
            phi0, phi1 = q[c, k], q[o, k]
            delta = phi1 - phi0
            g0 = 2.0 * np.einsum("fa,fa->f", gq[c, k], d0)
            s = g0 - delta
            eps = 1e-8 * (np.abs(phi0) + np.abs(phi1)) + 1e-30
            beta = np.abs(s - delta) / (np.abs(s) + np.abs(delta) + eps)
            r = np.clip(s * delta / (delta * delta + eps * eps), -2.0, 2.0)
            vals = [np.abs(g0), np.abs(delta), beta, np.abs(s - delta)]
            for j, v in enumerate(vals):
                np.maximum.at(acc_max[j], c, v)
            np.minimum.at(acc_min, c, r)
            np.add.at(sum_beta, c, beta)
            np.add.at(sum_dl, c, np.abs(delta))
            np.add.at(cnt, c, 1.0)
        del stats
        scale = np.abs(q[:, k]) + sum_dl / cnt + 1e-8
        f = np.stack([acc_max[0] / scale, acc_max[1] / scale, acc_max[2], sum_beta / cnt, acc_min,
                      acc_max[3] / scale], 1)
        out[:, 6 * k:6 * k + 6] = np.clip(f, -8.0, 8.0)
    return out


# ------------------------------------------------------------------ network
def unpack(theta):
    t = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = t[o:o + N_H * N_IN].reshape(N_H, N_IN); o += N_H * N_IN
    b1 = t[o:o + N_H]; o += N_H
    W2 = t[o:o + N_H * N_H].reshape(N_H, N_H); o += N_H * N_H
    b2 = t[o:o + N_H]; o += N_H
    W3 = t[o:o + N_H]; o += N_H
    b3 = t[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3, [b3]])


def xavier_init(seed):
    """Seeded Xavier-uniform weights, zero biases (an input of the method)."""
    rng = np.random.default_rng(seed)

    def u(fan_out, fan_in):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-a, a, size=(fan_out, fan_in))
    return pack(u(N_H, N_IN), np.zeros(N_H), u(N_H, N_H), np.zeros(N_H), u(1, N_H)[0], 0.0)


def forward(params, X, bf16=False):
    W1, b1, W2, b2, W3, b3 = unpack(params)
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    Xb = r(X)
    Z1 = Xb @ r(W1).T + b1
    H1 = np.tanh(Z1)
    Z2 = r(H1) @ r(W2).T + b2
    H2 = np.tanh(Z2)
    z3 = H2 @ W3 + b3
    th = 1.0 / (1.0 + np.exp(-z3))
    return th, (Xb, H1, H2)


def loss_and_grad(params, X, y, bf16=False):
    """Mean binary cross entropy and its gradient (chain rule, by hand)."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    th, (Xb, H1, H2) = forward(params, X, bf16)
    n = X.shape[0]
    tc = np.clip(th, 1e-12, 1 - 1e-12)
    loss = -np.mean(y * np.log(tc) + (1 - y) * np.log(1 - tc))
    g3 = (th - y) / n                        # dL/dz3 of sigmoid + BCE
    dW3 = H2.T @ g3
    db3 = g3.sum()
    d2 = np.outer(g3, W3) * (1 - H2 * H2)    # dL/dZ2
    d2b = r(d2)
    H1b = r(H1)
    dW2 = d2b.T @ H1b
    db2 = d2.sum(0)
    d1 = (d2b @ r(W2)) * (1 - H1 * H1)       # dL/dZ1
    d1b = r(d1)
    dW1 = d1b.T @ Xb
    db1 = d1.sum(0)
    return loss, pack(dW1, db1, dW2, db2, dW3, db3)


def adam_step(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba): returns (params, m, v); t counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
