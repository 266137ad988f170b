"""Per-cell evaluation counters (chem_eval_counters) on the GPU through the C
ABI, against the oracle's counts of the same evaluations: Jacobians (one per
step start) and right-hand sides (one per step start, two new-point stages
per attempt, n more per forward-difference Jacobian).

On every cell whose accepted/rejected step counts equal the oracle's, n_jac
and n_fev must equal the oracle's exactly (at most 0.1% of cells, rounded up,
may take another step sequence, as in the parity tests). Chained steps add up
the counts, mapped zonal cells get 0, and with the counters switched off no
integration writes them; a call with more cells than they hold is refused.
"""
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2112_05834_amd import chem, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NCPU = max(1, min(16, os.cpu_count() or 1))


def _to(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _counts(S, x, dt):
    n = x.shape[0]
    nj = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    nf = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    S.eval_counters(nj, nf)
    r = S.integrate(_to(x), dt)
    torch.cuda.synchronize()
    S.eval_counters(None, None)
    return r.n_acc.cpu().numpy(), r.n_rej.cpu().numpy(), r.status.cpu().numpy(), nj.cpu().numpy(), nf.cpu().numpy()


def _check(got, ref):
    na, nr, st, nj, nf = got
    ona, onr, ost, onj, onf = ref
    assert np.array_equal(st, ost)
    same = (na == ona) & (nr == onr)
    assert (~same).sum() <= max(1, int(1e-3 * len(same)))
    assert np.array_equal(nj[same], onj[same]) and np.array_equal(nf[same], onf[same])
    assert (nj > 0).all() and (nf > nj).all()
    return int(same.sum())


@pytest.mark.parametrize("wl_name,cells,opts", [
    ("spray54_262144", 256, {}),                                    # per-wave kernel, n = 55
    ("spray54_262144", 96, {"jacobian": chem.JAC_FD}),              # n more f per Jacobian
    ("spray54_262144", 96, {"scheme": chem.ROS4}),
    ("large160_524288", 24, {}),                                    # workgroup kernel, n = 161
    ("large160_524288", 8, {"jacobian": chem.JAC_FD, "state": chem.STATE_NO_BATH}),
])
def test_eval_counters_match_oracle(tmp_path, wl_name, cells, opts):
    print("counters", wl_name, cells, opts, flush=True)
    wl, mech, path, phi = synth.workload_inputs(wl_name, str(tmp_path), 4096)
    x = phi[synth.sample_indices(phi.shape[0], cells, 77)]
    S = chem.Solver(chem.Mechanism(path), chem.default_opts(schedule=chem.PERSISTENT, **opts), device=0)
    got = _counts(S, x, wl.dt)
    okw = {"scheme": opts.get("scheme", chem.RODAS3), "jacobian": opts.get("jacobian", chem.JAC_ANALYTICAL),
           "state": opts.get("state", chem.STATE_FULL)}
    ref = O.Mech(path).integrate(x, wl.dt, n_threads=NCPU, counts=True, **okw)
    same = _check(got, (ref[2], ref[3], ref[4], ref[5], ref[6]))
    print("%s: %d/%d cells with the oracle's counts" % (wl_name, same, cells), flush=True)


def test_eval_counters_steps_zonal_and_off(tmp_path):
    wl, mech, path, phi = synth.workload_inputs("spray54_262144", str(tmp_path), 4096)
    x = _to(phi[:512])
    S = chem.Solver(chem.Mechanism(path), chem.default_opts(schedule=chem.PERSISTENT), device=0)
    n = x.shape[0]
    # two chained steps add up the counts of two single steps
    nj = torch.zeros(n, dtype=torch.int32, device=DEV)
    nf = torch.zeros(n, dtype=torch.int32, device=DEV)
    S.eval_counters(nj, nf)
    r1 = S.integrate(x, wl.dt, h_io=False)
    torch.cuda.synchronize()
    j1, f1 = nj.clone(), nf.clone()
    S.integrate(r1.phi.clone(), wl.dt, h_io=False)
    torch.cuda.synchronize()
    j2, f2 = nj.clone(), nf.clone()
    out = torch.empty_like(x)
    S.integrate_steps(x, wl.dt, 2, h_io=False, out=out)
    torch.cuda.synchronize()
    assert torch.equal(nj, j1 + j2) and torch.equal(nf, f1 + f2)
    # switched off: nothing is written
    S.eval_counters(None, None)
    nj.fill_(-7)
    S.integrate(x, wl.dt, h_io=False)
    S.integrate_steps(x, wl.dt, 2, h_io=False, out=out)
    torch.cuda.synchronize()
    assert (nj == -7).all()
    # a call with more cells than the counters hold is refused before any work
    small = torch.full((16,), -7, dtype=torch.int32, device=DEV)
    S.eval_counters(small, None)
    with pytest.raises(chem.ChemError):
        S.integrate(x, wl.dt, h_io=False)
    with pytest.raises(chem.ChemError):
        S.integrate_steps(x, wl.dt, 2, h_io=False, out=out)
    torch.cuda.synchronize()
    assert (small == -7).all()
    S.eval_counters(None, None)
    # zonal mapping: mapped cells are not integrated and count 0
    amb = synth.generate_states(mech, 256, 6.0e6, "ambient", 106)
    c, yf, yo = synth.bilger_streams(mech)
    S.zone_config(c, yf, yo, 1e-6, 1.0)
    S.eval_counters(nj, nf)
    nj.fill_(-7)
    nf.fill_(-7)
    r, m = S.integrate_zonal(_to(amb), wl.dt)
    torch.cuda.synchronize()
    S.eval_counters(None, None)
    mapped = m.cpu().numpy() > 0
    a, b = nj.cpu().numpy()[:256], nf.cpu().numpy()[:256]
    na = r.n_acc.cpu().numpy()
    assert mapped.any() and (~mapped).any()
    assert (a[mapped] == 0).all() and (b[mapped] == 0).all()
    assert (a[~mapped] == na[~mapped]).all() and (b[~mapped] > a[~mapped]).all()
