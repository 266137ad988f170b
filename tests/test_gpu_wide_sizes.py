"""The workgroup-per-cell path across its range of state sizes (64 < n <= 256),
on the GPU through the C ABI, against the CPU oracle.

The sizes cover every count of row slots per lane (a lane holds physical rows
l + 64 s: two slots up to n = 128, three up to 192, four up to 256), the
largest size, and LU tail panels of width 1, 4, 5, 8, 9 and a full 12:

  n =  65  two slots, tail 5          n = 192  three slots, full last panel
  n =  97  tail 1                     n = 193  four slots, tail 1
  n = 128  two slots, tail 8          n = 233  tail 5
  n = 129  three slots, tail 9        n = 256  the largest size, tail 4

* blocked LU: pivots, info and factors bit-identical to the oracle's
  unblocked LU on random matrices, matrices whose every pivot is the current
  last row, a zero pivot in the middle, and M = g I - J of the mechanism;
  solves rel 1e-10;
* integration at n = 129, 193 and 256: the parity bar of the other tests
  (at most one cell, 0.1% rounded up, on another step sequence), plain and
  persistent schedules bit-identical.
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


def _mech(tmp_path, ns):
    mech = synth.generate_mechanism(ns, 3 * ns, ns // 4, ns // 10, 3000 + ns, ea_by_class=True)
    path = synth.write_mech(mech, str(tmp_path / ("m%d.mech" % ns)))
    return mech, path


def _last_row_pivots(rng, n):
    """P L U with |l| <= 1/2 below L's unit diagonal and P placing L's row k
    at the last row still uneliminated at every step k: partial pivoting then
    takes its pivot from the last row at every step."""
    L = np.tril(0.5 * rng.uniform(-1.0, 1.0, size=(n, n)), -1) + np.eye(n)
    U = np.triu(rng.uniform(-1.0, 1.0, size=(n, n)), 1) + np.diag(2.0 + rng.uniform(0.0, 1.0, size=n))
    arr = np.arange(n)
    for k in range(n - 2, -1, -1):
        arr[k], arr[n - 1] = arr[n - 1], arr[k]
    return L[arr] @ U


@pytest.mark.parametrize("ns", [64, 96, 127, 128, 191, 192, 232, 255])
def test_wide_lu_every_size(tmp_path, ns):
    mech, path = _mech(tmp_path, ns)
    n = ns + 1
    S = chem.Solver(chem.Mechanism(path), device=0)
    rng = np.random.Generator(np.random.PCG64(500 + ns))
    A = np.empty((6, n, n))
    A[0] = rng.normal(size=(n, n)) + 2.0 * np.eye(n)
    A[1] = rng.normal(size=(n, n))                     # no diagonal help: interchanges at most steps
    A[2] = _last_row_pivots(rng, n)
    A[3] = rng.normal(size=(n, n))
    A[3][:, n // 2] = 0.0                              # zero pivot in the middle: info = n // 2 + 1
    A[4] = np.round(rng.normal(size=(n, n)))           # many ties between candidates
    phi = synth.generate_states(mech, 1, 6.0e6, "bimodal", 4000 + ns)
    y = np.concatenate([[phi[0, 0]], phi[0, 2:]])
    A[5] = np.eye(n) / (0.5 * 1e-7) - O.Mech(path).jac(phi[0, 1], y)
    b = rng.normal(size=(6, n))
    Ag, piv, info, bg = S.lu_batch(_to(A), _to(b))
    torch.cuda.synchronize()
    Ag, piv, info, bg = Ag.cpu().numpy(), piv.cpu().numpy(), info.cpu().numpy(), bg.cpu().numpy()
    for k in range(6):
        LU, pr, inf = O.lu(A[k])
        assert info[k] == inf, (n, k)
        assert np.array_equal(piv[k], pr), (n, k)
        assert np.array_equal(Ag[k], LU), (n, k, np.nanmax(np.abs(Ag[k] - LU)))
        if inf == 0:
            x = O.lu_solve(LU, pr, b[k])
            assert np.max(np.abs(bg[k] - x)) <= 1e-10 * np.max(np.abs(x)), (n, k)
    assert (piv[2][:-1] == n - 1).all()
    assert info[3] == n // 2 + 1
    print("n=%d: factors of 6 matrices bit-identical to the oracle's" % n, flush=True)


def _run(S, x, dt):
    h = torch.zeros(x.shape[0], dtype=torch.float64, device=DEV)
    r = S.integrate(x, dt, h_io=h)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (r.phi, h, r.n_acc, r.n_rej, r.status)]


@pytest.mark.parametrize("ns", [128, 192, 255])
def test_wide_integrate_every_slot_count(tmp_path, ns):
    mech, path = _mech(tmp_path, ns)
    phi = synth.generate_states(mech, 32, 6.0e6, "bimodal", 4000 + ns)
    dt = 1e-6
    S = chem.Solver(chem.Mechanism(path), chem.default_opts(schedule=chem.PLAIN), device=0)
    plain = _run(S, _to(phi), dt)
    S.set_opts(chem.default_opts(schedule=chem.PERSISTENT))
    pers = _run(S, _to(phi), dt)
    for u, v in zip(plain, pers):
        assert np.array_equal(u.view(np.uint8), v.view(np.uint8))
    ref, h, na, nr_, st = O.Mech(path).integrate(phi, dt, n_threads=NCPU)
    gphi, _, gna, gnr, gst = plain
    assert np.array_equal(gst, st)
    same = (gna == na) & (gnr == nr_)
    assert (~same).sum() <= 1, "%d of %d cells took another step sequence" % ((~same).sum(), len(same))
    dT = np.abs(gphi[:, 0] - ref[:, 0])
    dY = np.abs(gphi[:, 2:] - ref[:, 2:])
    tolY = 1e-10 + 1e-6 * np.abs(ref[:, 2:])
    assert not (same & (dT > 1e-8 * np.abs(ref[:, 0]))).any()
    assert not (same[:, None] & (dY > tolY)).any()
    assert np.all(dT[~same] <= 1e-5 * np.abs(ref[~same, 0]))
    assert np.all(dY[~same] <= 10 * tolY[~same])
    assert np.array_equal(gphi[:, 1], phi[:, 1])
    print("n=%d: %d/%d cells on the oracle's step sequence, substeps %d..%d" %
          (ns + 1, same.sum(), len(same), (na + nr_).min(), (na + nr_).max()), flush=True)
