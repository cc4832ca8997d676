"""Oracle: float64 CPU reference of the learned-initial-guess network.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``). The network is not in
the paper; its parity with the GPU kernels is pinned here by central finite
differences of this float64 reference and by a direct loop evaluation of one
convolution, and the GPU forward/backward is compared against it.

Architecture (channels-last tensors [B][32^3][C], voxel index (z*32+y)*32+x):
  c1 16->16 @32 relu, avgpool 2, c2 16->32 @16 relu, avgpool 2,
  c3 32->64 @8 relu, c4 64->64 @8 relu, nearest up 2 and concat [up, c2],
  c5 96->32 @16 relu, nearest up 2 and concat [up, c1], c6 48->16 @32 relu,
  c7 16->16 @32 linear; loss = mean over the first 6 output channels of the
  squared difference to the target. Every convolution is 3x3x3, stride 1,
  zero padding 1, out[v][co] = b[co] + sum_{tap, ci} in[v + off(tap)][ci] W[tap][ci][co]
  with tap = 9 (dz+1) + 3 (dy+1) + (dx+1). Parameters are one flat vector,
  layer by layer W[27][Cin][Cout] then b[Cout].
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

SIDE = 32
LAYERS = ((16, 16), (16, 32), (32, 64), (64, 64), (96, 32), (48, 16), (16, 16))
USED = 6


def split_params(p):
    """Flat parameter vector -> [(W [27][Cin][Cout], b [Cout])] (views)."""
    out, off = [], 0
    for cin, cout in LAYERS:
        w = p[off: off + 27 * cin * cout].reshape(27, cin, cout)
        off += 27 * cin * cout
        b = p[off: off + cout]
        off += cout
        out.append((w, b))
    assert off == len(p)
    return out


def num_params() -> int:
    return sum(27 * a * b + b for a, b in LAYERS)


def _conv(x, w, b):
    """x [B][C][D][D][D]; w [27][Cin][Cout] -> conv3d weight [Cout][Cin][3][3][3]."""
    cin, cout = w.shape[1], w.shape[2]
    wt = w.permute(2, 1, 0).reshape(cout, cin, 3, 3, 3)
    return F.conv3d(x, wt, b, padding=1)


def forward(p, X):
    """p: flat float64 tensor; X: [B][32^3][16] -> Y [B][32^3][16]."""
    B = X.shape[0]
    x = X.reshape(B, SIDE, SIDE, SIDE, -1).permute(0, 4, 1, 2, 3)
    (w1, b1), (w2, b2), (w3, b3), (w4, b4), (w5, b5), (w6, b6), (w7, b7) = split_params(p)
    a1 = F.relu(_conv(x, w1, b1))
    a2 = F.relu(_conv(F.avg_pool3d(a1, 2), w2, b2))
    a3 = F.relu(_conv(F.avg_pool3d(a2, 2), w3, b3))
    a4 = F.relu(_conv(a3, w4, b4))
    q2 = torch.cat([F.interpolate(a4, scale_factor=2, mode="nearest"), a2], dim=1)
    a5 = F.relu(_conv(q2, w5, b5))
    q1 = torch.cat([F.interpolate(a5, scale_factor=2, mode="nearest"), a1], dim=1)
    a6 = F.relu(_conv(q1, w6, b6))
    y = _conv(a6, w7, b7)
    return y.permute(0, 2, 3, 4, 1).reshape(B, SIDE ** 3, -1)


def loss(p, X, T):
    Y = forward(p, X)
    return ((Y[..., :USED] - T) ** 2).mean()


def loss_and_grad(params: np.ndarray, X: np.ndarray, T: np.ndarray):
    """float64 loss and gradient with respect to the flat parameters."""
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    L = loss(p, torch.tensor(np.asarray(X, dtype=np.float64)), torch.tensor(np.asarray(T, dtype=np.float64)))
    L.backward()
    return float(L.detach()), p.grad.numpy().copy()


def conv_direct(x, w, b):
    """Direct loop form of one convolution (for pinning the tap convention):
    x [D][D][D][Cin] channels-last, w [27][Cin][Cout], b [Cout]."""
    D = x.shape[0]
    out = np.tile(np.asarray(b, dtype=np.float64), (D, D, D, 1))
    xp = np.zeros((D + 2, D + 2, D + 2, x.shape[3]))
    xp[1:-1, 1:-1, 1:-1] = x
    for tap in range(27):
        dz, dy, dx = tap // 9 - 1, (tap // 3) % 3 - 1, tap % 3 - 1
        sl = xp[1 + dz: 1 + dz + D, 1 + dy: 1 + dy + D, 1 + dx: 1 + dx + D]
        out += sl @ w[tap]
    return out
