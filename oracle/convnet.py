"""Learned initial guess of the stage solves: the definition of the network, its
training loss and optimiser, in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

This part is not in the paper: the paper starts every PCG solve from the zero
vector (Sec. 6).  The addition predicts the solution X_j of stage j from its
last four values H1..H4 (newest first) on the grid of free coefficients:

    D0 = H1, D1 = H1 - H2, D2 = H1 - 2 H2 + H3, D3 = H1 - 3 H2 + 3 H3 - H4
                                           (backward differences)
    E     = D0 + D1 + D2 + D3 = 4 H1 - 6 H2 + 4 H3 - H4
                                           (the cubic through the four values,
                                            evaluated one step ahead)
    s_c   = RMS(D_c)                       (1 when D_c = 0)
    guess = E + s_3 * net(D0/s_0, D1/s_1, D2/s_2, D3/s_3)

``net`` is three 3x3x3 cross-correlations, channels 4 -> 32 -> 32 -> 1, with a
bias each and ReLU after the first two, every layer zero-padded by one point
at the grid boundary (the homogeneous Dirichlet data).  Parameter vector
(32,033 values), tap-major: W1[27][4][32] b1[32] W2[27][32][32] b2[32]
W3[27][32][1] b3[1], tap t = 9 kz + 3 ky + kx, weight W[t][ci][co] applied to
input channel ci at offset (kx-1, ky-1, kz-1).  Grids are arrays [z][y][x].

Training loss: the mean squared difference between net(D/s) and the
normalised correction (X - E)/s_3 over the target boxes of a batch of crops
(box b = origin_b + 3 + [0, S-6)^3 per axis), the net evaluated on the whole
grid.  Optimiser: Adam with bias correction (Kingma and Ba, 2015).

Library primitives used as steps: torch.nn.functional.conv3d and autograd.
"""
import numpy as np
import torch
import torch.nn.functional as F

NPARAM = 27 * 4 * 32 + 32 + 27 * 32 * 32 + 32 + 27 * 32 + 1
LAYERS = ((4, 32), (32, 32), (32, 1))


def unpack(params):
    """Flat tap-major vector -> [(W [co][ci][kz][ky][kx], b [co]) x 3] (torch FP64)."""
    p = torch.as_tensor(np.asarray(params, dtype=np.float64)).reshape(-1)
    if p.numel() != NPARAM:
        raise ValueError(f"need {NPARAM} parameters")
    out, o = [], 0
    for ci, co in LAYERS:
        w = p[o:o + 27 * ci * co].reshape(3, 3, 3, ci, co)      # [kz][ky][kx][ci][co]
        o += 27 * ci * co
        b = p[o:o + co]
        o += co
        out.append((w.permute(4, 3, 0, 1, 2).contiguous(), b.clone()))
    return out


def pack(layers):
    """Inverse of ``unpack``."""
    parts = []
    for (w, b) in layers:
        w = torch.as_tensor(w, dtype=torch.float64)
        parts.append(w.permute(2, 3, 4, 1, 0).reshape(-1))
        parts.append(torch.as_tensor(b, dtype=torch.float64).reshape(-1))
    return torch.cat(parts).numpy()


def net_apply(layers, x):
    """x: [B][4][Z][Y][X] -> [B][Z][Y][X], zero padding per layer."""
    h = x
    for i, (w, b) in enumerate(layers):
        h = F.conv3d(h, w, b, padding=1)
        if i < 2:
            h = torch.relu(h)
    return h[:, 0]


def differences(H):
    H1, H2, H3, H4 = (np.asarray(h, dtype=np.float64) for h in H)
    return [H1, H1 - H2, H1 - 2.0 * H2 + H3, H1 - 3.0 * H2 + 3.0 * H3 - H4]


def extrapolation(H):
    H1, H2, H3, H4 = (np.asarray(h, dtype=np.float64) for h in H)
    return 4.0 * H1 - 6.0 * H2 + 4.0 * H3 - H4


def rms_scale(v):
    s = float(np.sqrt(np.mean(np.asarray(v, dtype=np.float64) ** 2)))
    return s if s > 0.0 else 1.0


def features(H, grid):
    """Net input [4][Z][Y][X] = D_c / s_c, and the output scale s_3."""
    D = differences(H)
    sc = [rms_scale(d) for d in D]
    return np.stack([D[c].reshape(grid) / sc[c] for c in range(4)]), sc[3]


def net_fields(params, H, grid):
    """net(D/s) on the grid (Z, Y, X) and s_3; H: 4 flat vectors in co-lex order."""
    x, s3 = features(H, grid)
    with torch.no_grad():
        return net_apply(unpack(params), torch.as_tensor(x)[None])[0].numpy(), s3


def learned_guess(params, H, grid):
    """E + s_3 net(D/s), flat co-lex vector."""
    out, s3 = net_fields(params, H, grid)
    return extrapolation(H) + s3 * out.reshape(-1)


def crops(H, X, grid, origins, S):
    """Training crops: in [nb][4][S][S][S] = D_c/s_c (zero outside the grid) and
    tgt [nb][S-6]^3 = (X - E)/s_3 on the crop interior; origins [nb] of (x, y, z)."""
    fields, s3 = features(H, grid)
    Z, Y, Xn = grid
    corr = ((np.asarray(X, dtype=np.float64) - extrapolation(H)) / s3).reshape(grid)
    pad = S
    fp = np.zeros((4, Z + 2 * pad, Y + 2 * pad, Xn + 2 * pad))
    fp[:, pad:pad + Z, pad:pad + Y, pad:pad + Xn] = fields
    ins, tgts = [], []
    T = S - 6
    for (ox, oy, oz) in origins:
        ins.append(fp[:, pad + oz:pad + oz + S, pad + oy:pad + oy + S, pad + ox:pad + ox + S])
        tgts.append(corr[oz + 3:oz + 3 + T, oy + 3:oy + 3 + T, ox + 3:ox + 3 + T])
    return np.stack(ins), np.stack(tgts)


def crop_loss(params, H, X, grid, origins, S, want_grad=True):
    """Mean squared error over the target boxes (net on the whole grid) and its
    gradient w.r.t. the flat parameter vector."""
    x, s3 = features(H, grid)
    fields = torch.as_tensor(x)[None]
    corr = torch.as_tensor(((np.asarray(X, dtype=np.float64) - extrapolation(H)) / s3).reshape(grid))
    p = torch.as_tensor(np.asarray(params, dtype=np.float64)).clone().requires_grad_(want_grad)
    layers, o = [], 0
    for ci, co in LAYERS:
        w = p[o:o + 27 * ci * co].reshape(3, 3, 3, ci, co).permute(4, 3, 0, 1, 2)
        o += 27 * ci * co
        b = p[o:o + co]
        o += co
        layers.append((w, b))
    out = net_apply(layers, fields)[0]
    T = S - 6
    err = []
    for (ox, oy, oz) in origins:
        sl = (slice(oz + 3, oz + 3 + T), slice(oy + 3, oy + 3 + T), slice(ox + 3, ox + 3 + T))
        err.append((out[sl] - corr[sl]).reshape(-1))
    loss = torch.mean(torch.cat(err) ** 2)
    if not want_grad:
        return float(loss.detach())
    loss.backward()
    return float(loss.detach()), p.grad.numpy().copy()


def adam_step(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v

