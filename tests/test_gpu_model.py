"""Learned cost model and binned queue on the GPU, through the C ABI.

* MLP forward and gradient against the BF16-emulating CPU oracle (the GPU
  rounds contraction operands to BF16 and accumulates in FP32, so only the
  FP32 summation order differs): norm-wise relative 1e-3.
* Octile edges and the binned queue order: exact (floats selected, integers
  permuted).
* Binned integration: phi, h, counters and status bit-identical to the
  unbinned schedules, with a trained model, with true-cost bins and on the
  non-finite-prediction fallback.

The timing test of what the bins gain is collected last, in its own file.
"""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as MO
from paper_2112_05834_amd import chem, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _to(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


@pytest.fixture(scope="module")
def spray(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("spray_model"))
    wl, mech, path, phi = synth.workload_inputs("spray54_262144", d, 16384)
    return wl, mech, path, phi


@pytest.fixture(scope="module")
def solver(spray):
    wl, mech, path, phi = spray
    return chem.Solver(chem.Mechanism(path), device=0)


def _random_model(seed, scale=0.3, n=1000):
    rng = _rng(seed)
    theta = rng.normal(0.0, scale, size=MO.N_PARAMS).astype(np.float32)
    X = rng.normal(0.0, 1.0, size=(n, 4)).astype(np.float32)
    T = rng.normal(1.0, 1.0, size=n).astype(np.float32)
    return theta, X, T


def _groups(v):
    p = MO.unflatten(v)
    return {k: np.asarray(p[k], dtype=np.float64).ravel() for k, _ in MO.SHAPES}


@pytest.mark.parametrize("n", [1, 31, 1000])
def test_predict_matches_bf16_oracle(solver, n):
    theta, X, T = _random_model(11 + n, n=n)
    solver.model_set(theta)
    y = solver.model_predict(_to(X)).cpu().numpy().astype(np.float64)
    ref, _ = MO.forward(MO.unflatten(theta.astype(np.float64)), X.astype(np.float64), "bf16")
    assert np.linalg.norm(y - ref) <= 1e-3 * np.linalg.norm(ref) + 1e-6
    ref64, _ = MO.forward(MO.unflatten(theta.astype(np.float64)), X.astype(np.float64), "fp64")
    assert np.linalg.norm(y - ref64) <= 3e-2 * np.linalg.norm(ref64) + 1e-6


@pytest.mark.parametrize("n", [32, 1000, 5000])
def test_gradient_matches_bf16_oracle(solver, n):
    theta, X, T = _random_model(5 + n, n=n)
    solver.model_set(theta)
    loss, g = solver.model_grad(_to(X), _to(T))
    g = g.cpu().numpy().astype(np.float64)
    loss = float(loss.cpu().numpy()[0])
    p = MO.unflatten(theta.astype(np.float64))
    l16, g16 = MO.loss_and_grad(p, X.astype(np.float64), T.astype(np.float64), "bf16")
    ref = MO.flatten(g16)
    assert abs(loss - l16) <= 1e-4 * abs(l16)
    assert np.linalg.norm(g - ref) <= 1e-3 * np.linalg.norm(ref)
    # every parameter group separately (a transposed or misplaced block fails here)
    G, R = _groups(g), _groups(ref)
    for k in R:
        assert np.linalg.norm(G[k] - R[k]) <= 2e-3 * np.linalg.norm(R[k]) + 1e-7, k
    l64, g64 = MO.loss_and_grad(p, X.astype(np.float64), T.astype(np.float64), "fp64")
    assert np.linalg.norm(g - MO.flatten(g64)) <= 3e-2 * np.linalg.norm(MO.flatten(g64))


def test_normalisation_applied(solver):
    theta, X, T = _random_model(3, n=500)
    mu = np.array([0.5, -1.0, 2.0, 0.0], dtype=np.float32)
    sd = np.array([2.0, 0.5, 1.0, 4.0], dtype=np.float32)
    solver.model_set(theta, np.concatenate([mu, sd]))
    y = solver.model_predict(_to(X)).cpu().numpy().astype(np.float64)
    Xn = ((X - mu) / sd).astype(np.float32).astype(np.float64)
    ref, _ = MO.forward(MO.unflatten(theta.astype(np.float64)), Xn, "bf16")
    assert np.linalg.norm(y - ref) <= 1e-3 * np.linalg.norm(ref)


def test_training_reduces_loss_deterministic_and_roundtrips(solver, tmp_path):
    rng = _rng(17)
    n = 20000
    X = rng.normal(size=(n, 4)).astype(np.float32)
    T = (2.0 + np.sin(2 * X[:, 0]) + 0.5 * X[:, 1] ** 2 - 0.3 * X[:, 2]).astype(np.float32)
    Xg, Tg = _to(X), _to(T)
    o = chem.default_train_opts(epochs=20, batch=1024, lr=3e-3, seed=5)
    solver.model_train(Xg, Tg, o)
    loss, _ = solver.model_grad(Xg, Tg)
    loss = float(loss.cpu()[0])
    assert loss < 0.1 * float(np.var(T)), (loss, np.var(T))
    p1, n1, e1 = solver.model_get()
    # normalisation equals the sample statistics
    assert np.allclose(n1[:4], X.astype(np.float64).mean(axis=0), rtol=1e-5, atol=1e-6)
    assert np.allclose(n1[4:], X.astype(np.float64).std(axis=0), rtol=1e-5)
    # edges: ascending octiles of the training predictions
    pred = solver.model_predict(Xg).cpu().numpy()
    assert e1 is not None and np.all(np.diff(e1) >= 0)
    counts = np.bincount(MO.bin_index(pred, e1), minlength=8)
    assert counts.min() >= n // 8 - 2 and counts.max() <= n // 8 + 2
    # same seed, same weights, bit for bit
    solver.model_train(Xg, Tg, o)
    p2, n2, e2 = solver.model_get()
    assert np.array_equal(p1.view(np.uint32), p2.view(np.uint32)) and np.array_equal(e1, e2)
    # save / load
    f = str(tmp_path / "model.bin")
    solver.model_save(f)
    solver.model_set(np.zeros(MO.N_PARAMS, dtype=np.float32))
    solver.model_load(f)
    pred2 = solver.model_predict(Xg).cpu().numpy()
    assert np.array_equal(pred.view(np.uint32), pred2.view(np.uint32))


@pytest.mark.parametrize("n", [1, 7, 8, 100, 4097, 100003])
def test_octile_edges_and_order_exact(solver, n):
    rng = _rng(100 + n)
    c = rng.normal(size=n).astype(np.float32)
    c[: n // 3] = np.round(c[: n // 3] * 4) / 4          # many ties
    if n > 10:
        c[5] = -0.0
        c[6] = 0.0
    cg = _to(c)
    e = solver.bin_edges(cg)
    ref_e = MO.octile_edges(c.astype(np.float64))
    assert np.array_equal(e.astype(np.float64), ref_e)
    perm = solver.bin_order(cg, e).cpu().numpy()
    assert np.array_equal(perm, MO.binned_order(c.astype(np.float64), e.astype(np.float64)))
    if n > 10:
        c[n // 2] = np.nan
        perm = solver.bin_order(_to(c), e).cpu().numpy()
        assert np.array_equal(perm, np.arange(n))


def _run(S, x, dt, **opts):
    S.set_opts(chem.default_opts(**opts))
    h = torch.zeros(x.shape[0], dtype=torch.float64, device=DEV)
    r = S.integrate(x, dt, h_io=h)
    torch.cuda.synchronize()
    return [r.phi.cpu().numpy(), h.cpu().numpy(), r.n_acc.cpu().numpy(), r.n_rej.cpu().numpy(),
            r.status.cpu().numpy()]


def _bitsame(a, b):
    for u, v in zip(a, b):
        assert u.dtype == v.dtype and np.array_equal(u.view(np.uint8), v.view(np.uint8))


@pytest.fixture(scope="module")
def trained(spray):
    """A solver whose model is trained on the integrator's own log of a plain run."""
    wl, mech, path, phi = spray
    S = chem.Solver(chem.Mechanism(path), device=0)
    x = _to(phi)
    S.log_enable(phi.shape[0])
    ref = _run(S, x, wl.dt, schedule=chem.PLAIN)
    f, t = S.log_fetch(phi.shape[0])
    assert f.shape[0] == phi.shape[0]
    S.log_enable(0)
    S.model_train(f.contiguous(), t.contiguous(), chem.default_train_opts(epochs=8, batch=1024, seed=3))
    return S, x, ref


def test_binned_bit_identical_to_plain(trained, spray):
    wl = spray[0]
    S, x, ref = trained
    _bitsame(_run(S, x, wl.dt, schedule=chem.PERSISTENT), ref)
    out = _run(S, x, wl.dt, schedule=chem.PERSISTENT_BINNED)
    assert S.last_binning_used()
    _bitsame(out, ref)
    # bins sorted by the true cost
    cost = _to(np.log(np.maximum(ref[2] + ref[3], 1)).astype(np.float32))
    S.set_cost_override(cost)
    out = _run(S, x, wl.dt, schedule=chem.PERSISTENT_BINNED, queue_chunk=4)
    assert S.last_binning_used()
    _bitsame(out, ref)
    S.set_cost_override(None)
    # ragged count, cpw 1 of a smaller variant is not available for n = 55:
    # a ragged prefix instead
    m = 1237
    out = _run(S, x[:m].contiguous(), wl.dt, schedule=chem.PERSISTENT_BINNED)
    _bitsame(out, [a[:m] for a in ref])


def test_binned_chained_steps_in_graph(trained, spray):
    wl = spray[0]
    S, x, _ = trained
    m = 2048
    xs = x[:m].contiguous()
    S.set_opts(chem.default_opts(schedule=chem.PERSISTENT))
    seq = xs.clone()
    for _ in range(3):
        seq = S.integrate(seq, wl.dt, h_io=False).phi.clone()
    S.set_opts(chem.default_opts(schedule=chem.PERSISTENT_BINNED))
    out = torch.empty_like(xs)
    for rep in range(2):   # capture, then replay
        out.zero_()
        r = S.integrate_steps(xs, wl.dt, 3, h_io=False, out=out)
        torch.cuda.synchronize()
        assert torch.equal(r.phi, seq), rep


def test_binned_fallback_on_nonfinite_prediction(trained, spray):
    wl = spray[0]
    S, x, ref = trained
    p, nv, e = S.model_get()
    bad = p.copy()
    bad[MO.N_PARAMS - 1] = np.nan            # output bias -> every prediction NaN
    S.model_set(bad, nv, e)
    try:
        out = _run(S, x, wl.dt, schedule=chem.PERSISTENT_BINNED)
        assert not S.last_binning_used()
        _bitsame(out, ref)
    finally:
        S.model_set(p, nv, e)


def test_binning_without_model_uses_queue_order(spray):
    wl, mech, path, phi = spray
    S = chem.Solver(chem.Mechanism(path), device=0)
    x = _to(phi[:512])
    a = _run(S, x, wl.dt, schedule=chem.PERSISTENT_BINNED)
    assert not S.last_binning_used()
    _bitsame(a, _run(S, x, wl.dt, schedule=chem.PLAIN))
