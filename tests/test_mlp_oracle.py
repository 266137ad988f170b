"""Pins of the learned-cost-model oracle: finite differences, PyTorch's
bfloat16 conversion and Adam, and a brute-force stable sort."""
import numpy as np
import torch

from oracle import mlp_oracle as MO


def _params(seed=0, scale=0.3):
    rng = np.random.Generator(np.random.PCG64(seed))
    return MO.unflatten(rng.normal(0.0, scale, size=MO.N_PARAMS))


def test_parameter_count():
    assert MO.N_PARAMS == 4 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4545


def test_bf16_round_matches_torch():
    rng = np.random.Generator(np.random.PCG64(1))
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-30, 100), 10.0 ** rng.uniform(-30, 30, 500),
                        [0.0, -0.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 65504.0, np.inf, -np.inf]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    got = MO.bf16_round(x)
    assert np.array_equal(got, ref)
    assert np.isnan(MO.bf16_round([np.nan])[0])


def test_gradient_matches_finite_differences():
    p = _params(2)
    rng = np.random.Generator(np.random.PCG64(3))
    X = rng.normal(size=(37, 4))
    T = rng.normal(size=37)
    theta = MO.flatten(p)
    loss, g = MO.loss_and_grad(p, X, T, "fp64")
    gflat = MO.flatten(g)
    idx = rng.choice(MO.N_PARAMS, size=200, replace=False)
    for k in idx:
        e = np.zeros_like(theta)
        e[k] = 1e-6
        lp, _ = MO.loss_and_grad(MO.unflatten(theta + e), X, T, "fp64")
        lm, _ = MO.loss_and_grad(MO.unflatten(theta - e), X, T, "fp64")
        fd = (lp - lm) / 2e-6
        assert abs(fd - gflat[k]) <= 1e-6 * max(1.0, abs(gflat[k])) + 1e-8


def test_gradient_matches_torch_autograd():
    p = _params(4)
    rng = np.random.Generator(np.random.PCG64(5))
    X = rng.normal(size=(64, 4))
    T = rng.normal(size=64)
    loss, g = MO.loss_and_grad(p, X, T, "fp64")
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    x = torch.tensor(X)
    h1 = torch.relu(x @ tp["W1"].T + tp["b1"])
    h2 = torch.relu(h1 @ tp["W2"].T + tp["b2"])
    y = h2 @ tp["w3"] + tp["b3"][0]
    L = torch.mean((y - torch.tensor(T)) ** 2)
    L.backward()
    assert abs(L.item() - loss) < 1e-12 * abs(loss)
    for k in p:
        assert np.allclose(g[k], tp[k].grad.numpy(), rtol=1e-10, atol=1e-12)


def test_bf16_mode_close_to_fp64():
    p = _params(6, scale=0.2)
    rng = np.random.Generator(np.random.PCG64(7))
    X = rng.normal(size=(256, 4))
    T = rng.normal(size=256)
    l64, g64 = MO.loss_and_grad(p, X, T, "fp64")
    l16, g16 = MO.loss_and_grad(p, X, T, "bf16")
    a, b = MO.flatten(g64), MO.flatten(g16)
    assert np.linalg.norm(a - b) <= 3e-2 * np.linalg.norm(a)
    assert abs(l64 - l16) <= 1e-2 * abs(l64)


def test_adam_matches_torch():
    rng = np.random.Generator(np.random.PCG64(8))
    theta = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    w = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(size=50)
        theta, m, v = MO.adam_step(theta, g, m, v, t)
        w.grad = torch.tensor(g)
        opt.step()
        assert np.allclose(theta, w.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_octiles_and_binned_order():
    rng = np.random.Generator(np.random.PCG64(9))
    c = rng.normal(size=1000)
    e = MO.octile_edges(c)
    assert np.all(np.diff(e) >= 0)
    b = MO.bin_index(c, e)
    counts = np.bincount(b, minlength=8)
    assert counts.min() >= 124 and counts.max() <= 126
    order = MO.binned_order(c, e)
    # brute force: stable sort by descending bin
    ref = np.argsort(-b, kind="stable")
    assert np.array_equal(order, ref)
    assert sorted(order.tolist()) == list(range(1000))
    c[5] = np.nan
    assert np.array_equal(MO.binned_order(c, e), np.arange(1000))


def test_standardize():
    X = np.array([[1.0, 5.0, 2.0, 0.0], [3.0, 5.0, 4.0, 0.0]])
    mu, sd = MO.standardize_stats(X)
    assert np.allclose(mu, [2, 5, 3, 0]) and np.allclose(sd, [1, 1, 1, 1])


def test_features_special_values():
    phi = np.zeros((2, 5))
    phi[0] = [1500.0, 1e5, 1.0, 1.0, 1.0]          # log10 1 = 0 for every species
    phi[1] = [800.0, 1e5 * np.e, 1e-40, 1e-10, 1e-20]
    f = MO.features(phi, 1e-5)
    assert np.allclose(f[0], [0.0, 0.0, 0.0, 1.0], atol=1e-15)
    assert np.allclose(f[1], [-1.0, 1.0, (-30 - 10 - 20) / 3 / 10, 1.0], atol=1e-14)
