"""Pins of the float64 reference network (CPU): the convolution's tap
convention against a direct loop, and the autograd gradient against central
finite differences."""
import numpy as np
import pytest
import torch

from oracle import network


def _he_params(seed):
    rng = np.random.default_rng(seed)
    p = np.zeros(network.num_params())
    off = 0
    for cin, cout in network.LAYERS:
        n = 27 * cin * cout
        p[off: off + n] = rng.normal(scale=np.sqrt(2.0 / (27 * cin)), size=n)
        off += n
        p[off: off + cout] = rng.normal(scale=0.05, size=cout)
        off += cout
    return p


def test_conv_matches_direct_loop():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(5, 5, 5, 3))
    w = rng.normal(size=(27, 3, 4))
    b = rng.normal(size=4)
    ref = network.conv_direct(x, w, b)
    xt = torch.tensor(x).permute(3, 0, 1, 2)[None]
    got = network._conv(xt, torch.tensor(w), torch.tensor(b))[0].permute(1, 2, 3, 0).numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = _he_params(2)
    X = rng.normal(size=(1, network.SIDE ** 3, 16))
    X[..., 5:] = 0.0
    T = rng.normal(size=(1, network.SIDE ** 3, network.USED))
    L, g = network.loss_and_grad(p, X, T)
    # one weight and one bias of every layer, among entries with a gradient of
    # at least 1e-3 of the layer's largest (inputs 5..15 are zero, so their
    # weights have exactly zero gradient)
    idx, off = [], 0
    for cin, cout in network.LAYERS:
        for n in (27 * cin * cout, cout):
            seg = np.abs(g[off: off + n])
            cand = np.flatnonzero(seg >= 1e-3 * seg.max())
            idx.append(off + int(rng.choice(cand)))
            off += n
    Xt, Tt = torch.tensor(X), torch.tensor(T)
    # h = 1e-7: ReLU kinks crossed by the perturbation grow with h, round-off
    # grows with 1/h; 1e-5 relative leaves room for both
    for i in idx:
        h = 1e-7
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (float(network.loss(torch.tensor(pp), Xt, Tt)) - float(network.loss(torch.tensor(pm), Xt, Tt))) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * abs(g[i]), (i, fd, g[i])
