"""Reference of the design surrogate's network, for tests only.

Plain FP64 CPU computation of the same network the GPU kernels run: 3x3
convolutions with dilation d, periodic padding along phi (the last axis) and
zero padding along r, a leaky activation, a final 1x1 convolution.  Weights
are [cout][cin * 9] with the column index c*9 + ky*3 + kx (ky along r, kx
along phi, tap offset d*(k-1)).  With bf16=True every layer's input
activations and weights are first rounded to bfloat16 (nearest even), as the
GPU path feeds its matrix cores; products and sums stay FP64 here.

Nothing under paper_2501_07979_amd is imported; the functions take plain
numpy arrays.  Pinned by tests/test_surrogate_ref.py against brute-force
loops and finite differences.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x):
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as
    float64.  Written from the bfloat16 format: keep the top 16 bits of the
    IEEE single after adding half an ulp of the kept part (plus the tie bit)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def conv3x3(x, w, b, dil):
    """x [cin][B][H][W], w [cout][cin*9], b [cout] -> [cout][B][H][W]:
    out[o, b, y, j] = b[o] + sum_{c, ky, kx} w[o, c*9+ky*3+kx] *
    x[c, b, y + d(ky-1), (j + d(kx-1)) mod W], zero outside 0 <= y < H."""
    import torch
    x = torch.as_tensor(np.asarray(x, dtype=np.float64))
    cin, B, H, W = x.shape
    cout = w.shape[0]
    d = int(dil)
    xt = x.permute(1, 0, 2, 3)                                   # [B][cin][H][W]
    xt = torch.cat([xt[..., W - d:], xt, xt[..., :d]], dim=3)   # periodic in phi
    xt = torch.nn.functional.pad(xt, (0, 0, d, d))              # zero in r
    wt = torch.as_tensor(np.asarray(w, dtype=np.float64)).reshape(cout, cin, 3, 3)
    out = torch.nn.functional.conv2d(xt, wt, dilation=d)        # [B][cout][H][W]
    out = out + torch.as_tensor(np.asarray(b, dtype=np.float64))[None, :, None, None]
    return out.permute(1, 0, 2, 3).numpy()


def conv1x1(x, w, b):
    x = np.asarray(x, dtype=np.float64)
    return np.einsum("oc,cbhw->obhw", np.asarray(w, np.float64), x) + np.asarray(b, np.float64)[:, None, None, None]


def leaky(z, slope):
    return np.where(z > 0, z, slope * z)


def forward(x, layers, slope, bf16=False):
    """layers: list of (w, b, k, dil, act).  Returns the output and every
    layer's (input, pre-activation, output) for backward."""
    h = np.asarray(x, dtype=np.float64)
    trace = []
    for (w, b, k, dil, act) in layers:
        hin = bf16_round(h) if bf16 else h
        wq = bf16_round(w) if bf16 else np.asarray(w, np.float64)
        z = conv3x3(hin, wq, b, dil) if k == 3 else conv1x1(hin, wq, b)
        y = leaky(z, slope) if act else z
        trace.append((hin, wq, z, y))
        h = y
    return h, trace


def backward(dy, layers, trace, slope):
    """Gradients of sum(dy * output) with respect to every layer's weights
    and biases (at the operands forward used) and to the input, by the
    chain rule through torch's autograd on FP64 tensors."""
    import torch
    grads = []
    g = torch.as_tensor(np.asarray(dy, dtype=np.float64))
    for (w, b, k, dil, act), (hin, wq, z, y) in zip(reversed(layers), reversed(trace)):
        hin_t = torch.as_tensor(hin).requires_grad_(True)
        w_t = torch.as_tensor(wq).requires_grad_(True)
        b_t = torch.as_tensor(np.asarray(b, np.float64)).requires_grad_(True)
        cin, B, H, W = hin.shape
        cout = wq.shape[0]
        if k == 3:
            d = int(dil)
            xt = hin_t.permute(1, 0, 2, 3)
            xt = torch.cat([xt[..., W - d:], xt, xt[..., :d]], dim=3)
            xt = torch.nn.functional.pad(xt, (0, 0, d, d))
            zt = torch.nn.functional.conv2d(xt, w_t.reshape(cout, cin, 3, 3), dilation=d)
            zt = zt.permute(1, 0, 2, 3) + b_t[:, None, None, None]
        else:
            zt = torch.einsum("oc,cbhw->obhw", w_t, hin_t) + b_t[:, None, None, None]
        yt = torch.where(zt > 0, zt, slope * zt) if act else zt
        (yt * g).sum().backward()
        grads.append((w_t.grad.numpy(), b_t.grad.numpy()))
        g = hin_t.grad
    return list(reversed(grads)), g.numpy()
