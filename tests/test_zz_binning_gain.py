"""What the learned binning gains, timed on the GPU (collected last: the only
GPU test whose assertion rests on a timing).

On cells ordered by ascending true cost, the queue in index order starts the
longest cells last; longest-first bins, from the trained model's predictions
and from the true costs, finish sooner.
"""
import numpy as np
import pytest
import torch

from paper_2112_05834_amd import chem, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _to(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.fixture(scope="module")
def trained(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("spray_gain"))
    wl, mech, path, phi = synth.workload_inputs("spray54_262144", d, 16384)
    S = chem.Solver(chem.Mechanism(path), chem.default_opts(schedule=chem.PLAIN), device=0)
    x = _to(phi)
    S.log_enable(phi.shape[0])
    r = S.integrate(x, wl.dt, h_io=False)
    torch.cuda.synchronize()
    f, t = S.log_fetch(phi.shape[0])
    S.log_enable(0)
    S.model_train(f.contiguous(), t.contiguous(), chem.default_train_opts(epochs=8, batch=1024, seed=3))
    cost = (r.n_acc + r.n_rej).cpu().numpy()
    return wl, S, x, cost


def _time(S, x, dt, reps=3, **opts):
    S.set_opts(chem.default_opts(**opts))
    out = torch.empty_like(x)
    S.integrate(x, dt, h_io=False, out=out)
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        S.integrate(x, dt, h_io=False, out=out)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def test_binning_gain_on_cost_sorted_cells(trained):
    wl, S, x, cost = trained
    order = np.argsort(cost, kind="stable")
    xs = x[_to(order.astype(np.int64))].contiguous()
    t_queue = _time(S, xs, wl.dt, schedule=chem.PERSISTENT)
    t_binned = _time(S, xs, wl.dt, schedule=chem.PERSISTENT_BINNED)
    assert S.last_binning_used()
    S.set_cost_override(_to(np.log(np.maximum(cost[order], 1)).astype(np.float32)))
    t_true = _time(S, xs, wl.dt, schedule=chem.PERSISTENT_BINNED)
    S.set_cost_override(None)
    print("queue order %.2f ms, predicted bins %.2f ms, true-cost bins %.2f ms" % (t_queue, t_binned, t_true))
    assert t_binned < t_queue
    assert t_true < t_queue
