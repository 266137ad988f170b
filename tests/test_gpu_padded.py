"""State sizes that no kernel variant matches exactly: the per-wave kernel
runs them in the next larger compiled size (the species vectors, J and M
are zero-padded; the padding must stay inert), the workgroup kernel with a
leading dimension rounded up to 16. Right-hand side and Jacobian against
the oracle (rel 1e-9), integration against the oracle (tolerances of the
parity tests), plain and persistent schedules bit-identical.

  25 species -> n = 26, per-wave kernel of size 32 (species-major passes)
  40 species -> n = 41, per-wave kernel of size 55 (reaction-major passes)
 100 species -> n = 101, workgroup kernel, ld = 112
 143 species -> n = 144, workgroup kernel, ld = 144: the LU's last panel is
                a full 12 columns and no leading-dimension padding is left
 144 species -> n = 145, workgroup kernel, ld = 160: the LU's last panel has
                a single column (its index arithmetic is checked in bounds on
                the CPU by tests/test_wide_lu_bounds.py for every n)

At most one cell (0.1% rounded up) may take another step sequence than the
oracle's.
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


def _scaled(J, y):
    s = np.abs(y).copy()
    s[0] = max(s[0], 1.0)
    s[1:] = np.maximum(s[1:], 1e-8)
    return J * s[None, :] / s[:, None]


def _run(S, x, dt):
    h = torch.zeros(x.shape[0], dtype=torch.float64, device=DEV)
    r = S.integrate(x, dt, h_io=h)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (r.phi, h, r.n_acc, r.n_rej, r.status)]


@pytest.mark.parametrize("ns,nr,n3,nt", [(25, 90, 10, 3), (40, 160, 20, 6), (100, 450, 60, 15),
                                         (143, 600, 80, 20), (144, 600, 80, 20)])
def test_padded_state_sizes(tmp_path, ns, nr, n3, nt):
    mech = synth.generate_mechanism(ns, nr, n3, nt, 1000 + ns, ea_by_class=True)
    path = synth.write_mech(mech, str(tmp_path / ("m%d.mech" % ns)))
    phi = synth.generate_states(mech, 96, 6.0e6, "bimodal", 2000 + ns)
    dt = 1e-6
    M = O.Mech(path)
    S = chem.Solver(chem.Mechanism(path), chem.default_opts(schedule=chem.PLAIN), device=0)
    x = phi[:16]
    f, J = S.eval_rhs_jac(_to(x))
    torch.cuda.synchronize()
    f, J = f.cpu().numpy(), J.cpu().numpy()
    for c in range(x.shape[0]):
        y = np.concatenate([[x[c, 0]], x[c, 2:]])
        fr = M.rhs(x[c, 1], y)
        Jr = M.jac(x[c, 1], y)
        scale = np.abs(Jr).sum(axis=1) * np.maximum(np.abs(y), 1e-8).max() + np.abs(fr)
        assert np.all(np.abs(f[c] - fr) <= 1e-9 * np.abs(fr) + 1e-12 * scale), c
        A, B = _scaled(J[c], y), _scaled(Jr, y)
        rowmax = np.abs(B).max(axis=1, keepdims=True)
        assert np.all(np.abs(A - B) <= 1e-9 * np.abs(B) + 1e-12 * rowmax), c
    plain = _run(S, _to(phi), dt)
    S.set_opts(chem.default_opts(schedule=chem.PERSISTENT))
    pers = _run(S, _to(phi), dt)
    for u, v in zip(plain, pers):
        assert np.array_equal(u.view(np.uint8), v.view(np.uint8))
    ref, h, na, nr_, st = M.integrate(phi, dt, n_threads=NCPU)
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
    print("ns=%d: %d/%d cells on the oracle's step sequence, substeps %d..%d" %
          (ns, same.sum(), len(same), (na + nr_).min(), (na + nr_).max()), flush=True)
