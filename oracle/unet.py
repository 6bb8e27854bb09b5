"""FP64 CPU reference of the learned-guess U-Net (test infrastructure only).

Plain PyTorch CPU ops in float64, with autograd for the gradients: the same
architecture and parameter-vector layout as the GPU network, used to check
its forward pass and its hand-written backward pass.  Architecture: four
levels with c[0..3] channels; per level two 3^3 convolutions (periodic
padding) each followed by ReLU; 2x2x2 average pooling between encoder
levels; nearest x2 upsampling, concatenated [upsampled | skip] on the way up;
a 1x1 head; mean-square loss, optionally plus a weighted mean square of the
7-point periodic Laplacian of the error.  The input is zero-padded to 16
channels.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

LAYERS = ("e0a", "e0b", "e1a", "e1b", "e2a", "e2b", "e3a", "e3b", "d2a", "d2b", "d1a", "d1b", "d0a", "d0b")


def layer_shapes(c, out_ch):
    """[(name, cin, cout)] of the 3^3 convolutions, then the head (c0 -> out_ch)."""
    io = [(16, c[0]), (c[0], c[0]), (c[0], c[1]), (c[1], c[1]), (c[1], c[2]), (c[2], c[2]), (c[2], c[3]),
          (c[3], c[3]), (c[3] + c[2], c[2]), (c[2], c[2]), (c[2] + c[1], c[1]), (c[1], c[1]),
          (c[1] + c[0], c[0]), (c[0], c[0])]
    return [(name, a, b) for name, (a, b) in zip(LAYERS, io)]


def param_count(c, out_ch):
    n = sum(co * 27 * ci + co for _, ci, co in layer_shapes(c, out_ch))
    return n + out_ch * c[0] + out_ch


def unpack(p, c, out_ch):
    """Parameter vector -> {name: (weight [cout, cin, 3, 3, 3], bias)}, head (w, b)."""
    out, off = {}, 0
    for name, ci, co in layer_shapes(c, out_ch):
        w = p[off:off + co * 27 * ci].reshape(co, 3, 3, 3, ci).permute(0, 4, 1, 2, 3)  # [co][dz][dy][dx][ci]
        off += co * 27 * ci
        b = p[off:off + co]
        off += co
        out[name] = (w, b)
    hw = p[off:off + out_ch * c[0]].reshape(out_ch, c[0])
    off += out_ch * c[0]
    hb = p[off:off + out_ch]
    return out, (hw, hb)


def _conv(x, wb):
    w, b = wb
    return F.relu(F.conv3d(F.pad(x, (1, 1, 1, 1, 1, 1), mode="circular"), w, b))


def forward(p, x, c, out_ch):
    """x: [in_ch, n, n, n] float64 (z, y, x order); returns [out_ch, n, n, n]."""
    L, (hw, hb) = unpack(p, c, out_ch)
    in_ch = x.shape[0]
    h = torch.zeros((1, 16) + tuple(x.shape[1:]), dtype=x.dtype)
    h[0, :in_ch] = x
    skips = []
    h = _conv(_conv(h, L["e0a"]), L["e0b"])
    skips.append(h)
    for k in (1, 2, 3):
        h = F.avg_pool3d(h, 2)
        h = _conv(_conv(h, L[f"e{k}a"]), L[f"e{k}b"])
        if k < 3:
            skips.append(h)
    for k in (2, 1, 0):
        h = torch.cat([F.interpolate(h, scale_factor=2, mode="nearest"), skips[k]], dim=1)
        h = _conv(_conv(h, L[f"d{k}a"]), L[f"d{k}b"])
    y = torch.einsum("oc,bczyx->bozyx", hw, h) + hb.view(1, -1, 1, 1, 1)
    return y[0]


def laplacian(d):
    """7-point periodic Laplacian of unit spacing of each channel of d [ch, n, n, n]."""
    return sum(torch.roll(d, s, dims=a) for a in (1, 2, 3) for s in (1, -1)) - 6.0 * d


def loss_and_grad(p_np, x_np, t_np, c, out_ch, lap_weight=0.0):
    """Loss mean((y-t)^2) + lap_weight * mean(Lap(y-t)^2) and its gradient with
    respect to the parameter vector."""
    p = torch.tensor(np.asarray(p_np, dtype=np.float64), requires_grad=True)
    x = torch.tensor(np.asarray(x_np, dtype=np.float64))
    t = torch.tensor(np.asarray(t_np, dtype=np.float64))
    y = forward(p, x, c, out_ch)
    loss = torch.mean((y - t) ** 2) + lap_weight * torch.mean(laplacian(y - t) ** 2)
    loss.backward()
    return float(loss.detach()), p.grad.detach().numpy()


def predict(p_np, x_np, c, out_ch):
    with torch.no_grad():
        return forward(torch.tensor(np.asarray(p_np, dtype=np.float64)),
                       torch.tensor(np.asarray(x_np, dtype=np.float64)), c, out_ch).numpy()
