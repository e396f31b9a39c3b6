"""CPU emulation of the BF16 training arithmetic of the learned-guess net (test
infrastructure): the crop loss and gradient with layer 2's MFMA operands rounded to
BF16 and everything else in FP64, to check the GPU's BF16 training kernels against
the same roundings, apart from the effect of the roundings themselves."""
import torch

from oracle import convnet as cn

# BF16 unit roundoff: a BF16 significand has 8 bits, so rounding to nearest moves a
# value by at most 2^-8 of itself
U_BF16 = 2.0 ** -8


def bf16_round(t):
    """Round to FP32, then to BF16 (to nearest even), as the MFMA path rounds its operands."""
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def bf16_crop_grad(params, H, X, grid, origins, S, rnd=bf16_round):
    """Loss and gradient of a crop batch computed crop by crop in FP64 on the CPU with
    exactly the roundings of BF16 training: layer 2's forward rounds a1 and W2, its
    backward-data pass d2 and W2, its backward-weight pass a1 and d2; everything else
    exact; rnd = identity gives the exact loss and gradient.  Independent of the GPU
    code: valid convolutions of torch on each crop, activations outside the grid
    zeroed as the crop formulation prescribes."""
    import torch.nn.functional as F
    from torch.nn.grad import conv3d_input, conv3d_weight
    layers = cn.unpack(params)
    (w1, b1), (w2, b2), (w3, b3) = layers
    ins, tgts = cn.crops(H, X, grid, origins, S)
    x = torch.as_tensor(ins)
    tgt = torch.as_tensor(tgts)[:, None]
    Z, Y, Xn = grid

    def mask(shift, size):
        m = torch.zeros(len(origins), 1, size, size, size, dtype=torch.float64)
        r = torch.arange(size)
        for b, (ox, oy, oz) in enumerate(origins):
            mz = ((oz + shift + r) >= 0) & ((oz + shift + r) < Z)
            my = ((oy + shift + r) >= 0) & ((oy + shift + r) < Y)
            mx = ((ox + shift + r) >= 0) & ((ox + shift + r) < Xn)
            m[b, 0] = (mz[:, None, None] & my[None, :, None] & mx[None, None, :]).double()
        return m

    a1 = torch.relu(F.conv3d(x, w1, b1)) * mask(1, S - 2)
    a2 = torch.relu(F.conv3d(rnd(a1), rnd(w2), b2)) * mask(2, S - 4)
    out = F.conv3d(a2, w3, b3)
    n = out.numel()
    loss = float(torch.mean((out - tgt) ** 2))
    d3 = 2.0 * (out - tgt) / n
    gw3, gb3 = conv3d_weight(a2, w3.shape, d3), d3.sum(dim=(0, 2, 3, 4))
    d2 = conv3d_input(a2.shape, w3, d3) * (a2 > 0)
    gw2, gb2 = conv3d_weight(rnd(a1), w2.shape, rnd(d2)), d2.sum(dim=(0, 2, 3, 4))
    d1 = conv3d_input(a1.shape, rnd(w2), rnd(d2)) * (a1 > 0)
    gw1, gb1 = conv3d_weight(x, w1.shape, d1), d1.sum(dim=(0, 2, 3, 4))
    return loss, cn.pack([(gw1, gb1), (gw2, gb2), (gw3, gb3)])
