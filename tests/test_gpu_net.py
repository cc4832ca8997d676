"""GPU checks of the learned-initial-guess kernels (BF16 MFMA convolutions,
backward passes, Adam) against the float64 CPU reference network, and of the
end-to-end learned guess. Marked `gpu`.

Tolerances: BF16 activations are rounded after every layer (8-bit mantissa,
relative step 2^-8), with FP32 accumulation; outputs must match the float64
reference within 3e-2 (relative L2), each layer's weight gradient within
5e-2 (relative L2). Element by element: max |y - y_ref| <= 8 * 2^-8 max |y_ref|
for the outputs and <= 16 * 2^-8 max |g_ref| for each layer's weight
gradient (seven layers of rounding forward, fourteen through the backward
pass, each at most half a step of 2^-8 relative, with the errors of a sum no
larger than the largest term's).
"""
import numpy as np
import pytest

from oracle import network
from paper_1808_00186_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1808_00186_amd import learned, petgem
    petgem.lib()
    return torch, petgem, learned


def _bf16_input(torch, B, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(B, network.SIDE ** 3, 16)).astype(np.float32)
    x[..., 5:] = 0.0
    xt = torch.tensor(x, device="cuda").to(torch.bfloat16)
    return xt, xt.float().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_mfma_layout_and_forward_match_reference(env):
    torch, petgem, _ = env
    net = petgem.Net(batch_max=2, seed=7)
    x, x64 = _bf16_input(torch, 2, 1)
    y = net.forward(x).cpu().numpy()
    p = net.params().astype(np.float64)
    ref = network.forward(torch.tensor(p), torch.tensor(x64)).numpy()
    err = _rel(y, ref)
    emax = float(np.abs(y - ref).max() / np.abs(ref).max())
    print(f"net forward rel err {err:.3e}, max element error {emax:.3e} of max |y|", flush=True)
    assert err <= 3e-2
    assert emax <= 8 * 2.0 ** -8


def test_gradients_match_reference(env):
    torch, petgem, _ = env
    net = petgem.Net(batch_max=2, seed=11)
    x, x64 = _bf16_input(torch, 2, 2)
    rng = np.random.default_rng(3)
    t = rng.normal(size=(2, network.SIDE ** 3, network.USED)).astype(np.float32) * 0.3
    loss, g = net.loss_grad(x, torch.tensor(t, device="cuda"))
    p = net.params().astype(np.float64)
    L, gref = network.loss_and_grad(p, x64, t.astype(np.float64))
    assert abs(loss - L) <= 1e-2 * abs(L)
    off = 0
    for li, (cin, cout) in enumerate(network.LAYERS):
        n = 27 * cin * cout
        ew = _rel(g[off: off + n], gref[off: off + n])
        eb = _rel(g[off + n: off + n + cout], gref[off + n: off + n + cout])
        gw, gw_ref = g[off: off + n], gref[off: off + n]
        em = float(np.abs(gw - gw_ref).max() / np.abs(gw_ref).max())
        print(f"layer {li} grad W rel {ew:.2e} b rel {eb:.2e}, W max element error {em:.2e} of max", flush=True)
        assert ew <= 5e-2 and eb <= 5e-2
        assert em <= 16 * 2.0 ** -8
        off += n + cout


def test_gradients_are_bitwise_reproducible(env):
    """The weight pass sums voxel splits in a fixed order: two evaluations of
    the same batch give identical gradients (batch 3 also exercises a batch
    that is not a power of two)."""
    torch, petgem, _ = env
    net = petgem.Net(batch_max=3, seed=13)
    x, _ = _bf16_input(torch, 3, 4)
    t = torch.tensor(np.random.default_rng(5).normal(size=(3, network.SIDE ** 3, network.USED)) * 0.3,
                     dtype=torch.float32, device="cuda")
    l1, g1 = net.loss_grad(x, t)
    l2, g2 = net.loss_grad(x, t)
    assert l1 == l2
    assert np.array_equal(g1, g2)


def test_learned_x0_many_matches_one_system_at_a_time(env):
    """Guesses of systems on different meshes from one network batch equal the
    per-system guesses bitwise (the forward pass has no cross-sample terms)."""
    torch, petgem, _ = env
    meshes = [synth.kuhn_mesh(8, -1000.0, 1000.0, 1), synth.kuhn_mesh(6, -1000.0, 1000.0, 2),
              synth.kuhn_mesh(8, -1000.0, 1000.0, 1)]
    models = [synth.config5_sample(30000 + k, m) for k, m in enumerate(meshes)]
    systems = [petgem.System.from_model(m) for m in models]
    srcs = [m.sources[0] for m in models]
    net = petgem.Net(batch_max=4, seed=17)
    g = 0.5
    many, bn_many = petgem.learned_x0_many(systems, net, srcs, g)
    for k, (S, src) in enumerate(zip(systems, srcs)):
        one, bn_one = petgem.learned_x0(S, net, [src], g)
        assert many[k].shape == (S.n_dof,)
        assert torch.isfinite(torch.view_as_real(many[k])).all()
        assert torch.equal(many[k], one[0])
        assert bn_many[k] == bn_one[0]
    with pytest.raises(petgem.PetgemError):
        petgem.learned_x0_many(systems * 2, net, srcs * 2, g)   # more systems than batch_max


def test_learned_guess_trains_and_solves(env):
    torch, petgem, learned = env
    mesh = synth.kuhn_mesh(8, -1000.0, 1000.0, 1)
    m0 = synth.config5_sample(10000, mesh)
    S = petgem.System.from_model(m0)
    opts = petgem.default_opts(rtol=1e-8)
    g = learned.pilot_scale(S, range(10000, 10008), mesh, opts)
    data = learned.generate(S, list(range(10000, 10096)), mesh, g, opts)
    assert np.all(np.isfinite(data.bnorm))
    net = petgem.Net(batch_max=16, seed=5)
    import time
    t0 = time.perf_counter()
    losses = learned.train(net, data, epochs=30, batch=16, lr=2e-3)
    print(f"learned: g {g:.3e} data {data.seconds:.1f} s, 30 epochs {time.perf_counter() - t0:.1f} s, "
          f"loss {losses[0]:.3e} -> {losses[-1]:.3e}", flush=True)
    assert losses[-1] < 0.85 * losses[0]
    res = learned.evaluate(S, net, list(range(20000, 20006)), mesh, g, opts)
    print(f"learned eval: zero {res.iters_zero} learned {res.iters_learned} fallback {res.fallback} "
          f"x0 res {np.round(res.x0_residual, 3)} rx diff {res.max_rx_diff:.1e}", flush=True)
    # same answer at the same tolerance, whatever the guess
    assert res.max_rx_diff <= 1e-6
    # the same seeds as one uneven batch, zero and learned guesses
    rb = learned.evaluate_batched(net, list(range(20000, 20006)), mesh, g, opts)
    print(f"batched eval: zero {rb.iters_zero} learned {rb.iters_learned} fallback {rb.fallback} "
          f"rx diff {rb.max_rx_diff:.1e}", flush=True)
    assert rb.max_rx_diff <= 1e-6
    for a, b in zip(rb.E_zero, res.E_zero):
        num = np.sqrt(np.sum(np.abs(a - b) ** 2, axis=-1))
        assert np.max(num / np.sqrt(np.sum(np.abs(b) ** 2, axis=-1))) <= 1e-6
