"""Pins of the learned-guess oracle (oracle/convnet.py) against brute force,
closed forms, finite differences and a library routine."""
import numpy as np
import pytest
import torch

from oracle import convnet as cn
from paper_2102_11536_amd.workloads import gnet_random_params


def _brute_net(params, x):
    """The net from the tap-major definition with explicit loops over points and
    taps (channels as small matrix products); x [4][Z][Y][X]."""
    p = np.asarray(params, dtype=np.float64)
    h = np.asarray(x, dtype=np.float64)
    o = 0
    for li, (ci, co) in enumerate(cn.LAYERS):
        W = p[o:o + 27 * ci * co].reshape(27, ci, co)
        o += 27 * ci * co
        b = p[o:o + co]
        o += co
        Z, Y, X = h.shape[1:]
        out = np.zeros((co, Z, Y, X))
        for z in range(Z):
            for y in range(Y):
                for xx in range(X):
                    acc = b.copy()
                    for t in range(27):
                        kz, ky, kx = t // 9, (t // 3) % 3, t % 3
                        zz, yy, xs = z + kz - 1, y + ky - 1, xx + kx - 1
                        if 0 <= zz < Z and 0 <= yy < Y and 0 <= xs < X:
                            acc += W[t].T @ h[:, zz, yy, xs]
                    out[:, z, y, xx] = acc
        h = np.maximum(out, 0.0) if li < 2 else out
    return h[0]


def test_net_matches_brute_force():
    rng = np.random.default_rng(3)
    params = gnet_random_params(7)
    x = rng.standard_normal((4, 3, 4, 5))
    ref = _brute_net(params, x)
    with torch.no_grad():
        got = cn.net_apply(cn.unpack(params), torch.as_tensor(x)[None])[0].numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_pack_unpack_roundtrip():
    params = gnet_random_params(1)
    assert np.array_equal(cn.pack(cn.unpack(params)), params)
    assert cn.NPARAM == 32033


def test_extrapolation_exact_for_cubics():
    # H1..H4 = q(0), q(-1), q(-2), q(-3): E = q(1) for every cubic q, not for a quartic
    rng = np.random.default_rng(0)
    c = rng.standard_normal((4, 10))
    q = lambda t: c[0] + c[1] * t + c[2] * t ** 2 + c[3] * t ** 3
    H = [q(0.0), q(-1.0), q(-2.0), q(-3.0)]
    assert np.allclose(cn.extrapolation(H), q(1.0), rtol=0, atol=1e-12)
    q4 = lambda t: t ** 4
    assert abs(cn.extrapolation([q4(0), q4(-1), q4(-2), q4(-3)]) - q4(1)) > 1.0


def test_guess_special_cases():
    rng = np.random.default_rng(1)
    grid = (3, 4, 5)
    H = [rng.standard_normal(60) for _ in range(4)]
    E = cn.extrapolation(H)
    assert np.allclose(cn.learned_guess(np.zeros(cn.NPARAM), H, grid), E, rtol=0, atol=1e-14)
    # only the output bias: guess = E + s_3 * b3 with s_3 = RMS(H1 - 3H2 + 3H3 - H4)
    p = np.zeros(cn.NPARAM)
    p[-1] = 0.25
    s3 = np.sqrt(np.mean((H[0] - 3 * H[1] + 3 * H[2] - H[3]) ** 2))
    assert np.allclose(cn.learned_guess(p, H, grid), E + 0.25 * s3, rtol=0, atol=1e-13)


def test_differences_sum_to_extrapolation():
    # Newton's backward form: E = D0 + D1 + D2 + D3
    rng = np.random.default_rng(11)
    H = [rng.standard_normal(30) for _ in range(4)]
    assert np.allclose(sum(cn.differences(H)), cn.extrapolation(H), rtol=0, atol=1e-13)


def test_crops_brute_force():
    rng = np.random.default_rng(2)
    grid = (7, 8, 9)
    n = 7 * 8 * 9
    H = [rng.standard_normal(n) for _ in range(4)]
    X = rng.standard_normal(n)
    S = 8
    origins = [(0, 1, -2), (-3, -3, -3), (2, 1, 0)]
    inp, tgt = cn.crops(H, X, grid, origins, S)
    D = [H[0], H[0] - H[1], H[0] - 2 * H[1] + H[2], H[0] - 3 * H[1] + 3 * H[2] - H[3]]
    sc = [np.sqrt(np.mean(d ** 2)) for d in D]
    E = 4 * H[0] - 6 * H[1] + 4 * H[2] - H[3]
    for b, (ox, oy, oz) in enumerate(origins):
        for (lz, ly, lx) in [(0, 0, 0), (3, 4, 5), (S - 1, S - 1, S - 1), (3, 3, 3)]:
            z, y, x = oz + lz, oy + ly, ox + lx
            ok = 0 <= z < 7 and 0 <= y < 8 and 0 <= x < 9
            i = x + 9 * (y + 8 * z)
            for c in range(4):
                assert np.isclose(inp[b, c, lz, ly, lx], D[c][i] / sc[c] if ok else 0.0, rtol=1e-13, atol=0)
        i = (ox + 3) + 9 * ((oy + 3) + 8 * (oz + 3))
        assert np.isclose(tgt[b, 0, 0, 0], (X[i] - E[i]) / sc[3], rtol=1e-13)


def test_crop_loss_gradient_finite_differences():
    rng = np.random.default_rng(4)
    grid = (8, 8, 8)
    n = 512
    H = [rng.standard_normal(n) for _ in range(4)]
    X = rng.standard_normal(n)
    params = gnet_random_params(5)
    origins = [(-1, 0, -2), (1, 2, 0)]
    S = 10
    loss, grad = cn.crop_loss(params, H, X, grid, origins, S)
    idx = [0, 100, 3455, 3456, 3470, 3488, 20000, 31135, 31136, 31168, 31500, 32032]
    h = 1e-6
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (cn.crop_loss(pp, H, X, grid, origins, S, want_grad=False)
              - cn.crop_loss(pm, H, X, grid, origins, S, want_grad=False)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])), (i, fd, grad[i])
    assert loss > 0


def test_crop_loss_is_mean_over_target_boxes():
    # a net that outputs exactly the target (zero loss) is not available, but with
    # all-zero parameters the loss is the mean of the squared normalised correction
    rng = np.random.default_rng(6)
    grid = (6, 7, 8)
    n = 6 * 7 * 8
    H = [rng.standard_normal(n) for _ in range(4)]
    X = rng.standard_normal(n)
    origins = [(0, 0, 0), (-3, -2, -3)]
    S = 8
    _, tgt = cn.crops(H, X, grid, origins, S)
    loss = cn.crop_loss(np.zeros(cn.NPARAM), H, X, grid, origins, S, want_grad=False)
    assert np.isclose(loss, np.mean(tgt ** 2), rtol=1e-13)


def test_adam_matches_torch():
    rng = np.random.default_rng(8)
    p0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) for _ in range(3)]
    t = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for k, g in enumerate(grads, start=1):
        opt.zero_grad()
        t.grad = torch.tensor(g)
        opt.step()
        p, m, v = cn.adam_step(p, m, v, g, k, 1e-2)
    assert np.allclose(p, t.detach().numpy(), rtol=0, atol=1e-12)


def test_bf16_emulation_without_rounding_is_the_oracle():
    """The crop-by-crop emulation of BF16 training (tests/gnet_emulation.py) with the
    rounding switched off reproduces the oracle's loss and gradient (whole-grid net,
    autograd): its crops, masks and explicit backward passes are right; with the
    rounding on it moves the gradient by a few BF16 units only."""
    from tests.gnet_emulation import U_BF16, bf16_crop_grad
    mf = (10, 9, 8)
    grid = (mf[2], mf[1], mf[0])
    rng = np.random.default_rng(6)
    n = int(np.prod(mf))
    H = [rng.standard_normal(n) * (1.0 + 0.1 * h) for h in range(4)]
    X = rng.standard_normal(n)
    S = 10
    org = [(-3, -3, -3), (mf[0] - 7, mf[1] - 7, mf[2] - 7), (0, 1, -2)]
    params = gnet_random_params(8)
    rl, rg = cn.crop_loss(params, H, X, grid, org, S)
    el, eg = bf16_crop_grad(params, H, X, grid, org, S, rnd=lambda t: t)
    assert abs(el - rl) <= 1e-13 * rl
    assert np.linalg.norm(eg - rg) <= 1e-13 * np.linalg.norm(rg)
    bl, bg = bf16_crop_grad(params, H, X, grid, org, S)
    e = np.linalg.norm(bg - rg) / np.linalg.norm(rg)
    assert 0.0 < e <= 4 * U_BF16
    assert abs(bl - rl) <= 4 * U_BF16 * rl
