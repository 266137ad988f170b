"""GPU parity through the C ABI: the HIP path against the CPU oracle on the
same seeded inputs, element by element.

Tolerances: T relative 1e-8, Y within 1e-10 + 1e-6 |Y| on cells whose
accepted/rejected step counts equal the oracle's; at most 0.1% of cells may
take a different step sequence (an accept/reject decision at err ~ 1 flipped by
last-bit differences of exp/log), and those must still agree within ten times
the integration tolerance.
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


def _compare_h(h_gpu, h_ref, same, what):
    """The proposed next substep (h_io out) on cells with the oracle's step
    sequence: the controller's factor goes as err^(-1/3), so last-bit
    differences of the error estimate move it far below 1e-6."""
    rel = np.abs(h_gpu - h_ref) / np.abs(h_ref)
    print("%s: max relative difference of h_io out %.2e" % (what, rel[same].max() if same.any() else 0.0))
    assert (h_ref > 0).all() and (rel[same] <= 1e-6).all()


def _compare(phi0, gpu, ref, counts_gpu, counts_ref, frac_diff=1e-3):
    na, nr = counts_gpu
    ona, onr = counts_ref
    same = (na == ona) & (nr == onr)
    n = len(same)
    assert (~same).sum() <= max(1, int(frac_diff * n)), "%d of %d cells took another step sequence" % ((~same).sum(), n)
    dT = np.abs(gpu[:, 0] - ref[:, 0])
    dY = np.abs(gpu[:, 2:] - ref[:, 2:])
    tolY = 1e-10 + 1e-6 * np.abs(ref[:, 2:])
    bad_T = same & (dT > 1e-8 * np.abs(ref[:, 0]))
    bad_Y = same[:, None] & (dY > tolY)
    assert not bad_T.any(), "T differs on %d cells, worst rel %.3e" % (bad_T.sum(), (dT / ref[:, 0]).max())
    assert not bad_Y.any(), "Y differs on %d entries, worst %.3e" % (bad_Y.sum(), (dY / tolY).max())
    if (~same).any():
        assert np.all(dT[~same] <= 10 * 1e-6 * np.abs(ref[~same, 0]))
        assert np.all(dY[~same] <= 10 * tolY[~same])
    assert np.array_equal(gpu[:, 1], phi0[:, 1])
    return int(same.sum())


@pytest.fixture(scope="module")
def tiny(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("tiny"))
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", d)
    return wl, mech, path, phi


@pytest.fixture(scope="module")
def spray(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("spray"))
    wl, mech, path, phi = synth.workload_inputs("spray54_262144", d)
    return wl, mech, path, phi


def _scaled(J, y):
    s = np.abs(y).copy()
    s[0] = max(s[0], 1.0)
    s[1:] = np.maximum(s[1:], 1e-8)
    return J * s[None, :] / s[:, None]


@pytest.mark.parametrize("which", ["tiny", "spray"])
def test_rhs_and_jacobian_match_oracle(which, tiny, spray):
    wl, mech, path, phi = tiny if which == "tiny" else spray
    idx = synth.sample_indices(phi.shape[0], 64, 21)
    x = phi[idx]
    S = chem.Solver(chem.Mechanism(path), device=0)
    f, J = S.eval_rhs_jac(_to(x))
    torch.cuda.synchronize()
    f, J = f.cpu().numpy(), J.cpu().numpy()
    M = O.Mech(path)
    for c in range(len(idx)):
        y = np.concatenate([[x[c, 0]], x[c, 2:]])
        fr = M.rhs(x[c, 1], y)
        Jr = M.jac(x[c, 1], y)
        scale = np.abs(Jr).sum(axis=1) * np.maximum(np.abs(y), 1e-8).max() + np.abs(fr)
        assert np.all(np.abs(f[c] - fr) <= 1e-9 * np.abs(fr) + 1e-12 * scale), c
        A, B = _scaled(J[c], y), _scaled(Jr, y)
        rowmax = np.abs(B).max(axis=1, keepdims=True)
        assert np.all(np.abs(A - B) <= 1e-9 * np.abs(B) + 1e-12 * rowmax), c


def test_lu_batch_matches_oracle(tiny, spray):
    for wl, mech, path, phi in (tiny, spray):
        S = chem.Solver(chem.Mechanism(path), device=0)
        n = mech.n_species + 1
        rng = np.random.Generator(np.random.PCG64(n))
        A = rng.normal(size=(40, n, n)) + 3.0 * np.eye(n)[None]
        b = rng.normal(size=(40, n))
        # also real integrator matrices at a few states
        M = O.Mech(path)
        for c in range(8):
            y = np.concatenate([[phi[c, 0]], phi[c, 2:]])
            A[c] = np.eye(n) / (0.5 * 1e-8) - M.jac(phi[c, 1], y)
        Ag, piv, info, bg = S.lu_batch(_to(A), _to(b))
        torch.cuda.synchronize()
        Ag, piv, info, bg = Ag.cpu().numpy(), piv.cpu().numpy(), info.cpu().numpy(), bg.cpu().numpy()
        assert (info == 0).all()
        for k in range(A.shape[0]):
            LU, pr, inf = O.lu(A[k])
            assert np.array_equal(piv[k], pr), k
            assert np.max(np.abs(Ag[k] - LU)) <= 1e-12 * np.max(np.abs(A[k])), k
            x = O.lu_solve(LU, pr, b[k])
            assert np.max(np.abs(bg[k] - x)) <= 1e-10 * np.max(np.abs(x)), k


def test_lu_batch_singular_info(tiny):
    wl, mech, path, phi = tiny
    S = chem.Solver(chem.Mechanism(path), device=0)
    n = mech.n_species + 1
    A = np.eye(n)[None].repeat(2, axis=0)
    A[1, 3, :] = 0.0
    A[1, :, 3] = 0.0
    _, piv, info, _ = S.lu_batch(_to(A))
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, 4]


def test_integrate_tiny_all_cells(tiny):
    wl, mech, path, phi = tiny
    S = chem.Solver(chem.Mechanism(path), device=0)
    r = S.integrate(_to(phi), wl.dt)
    torch.cuda.synchronize()
    ref, h, na, nr, st = O.Mech(path).integrate(phi, wl.dt, n_threads=NCPU)
    assert np.array_equal(r.status.cpu().numpy(), st)
    same = _compare(phi, r.phi.cpu().numpy(), ref, (r.n_acc.cpu().numpy(), r.n_rej.cpu().numpy()), (na, nr))
    print("tiny: %d/1024 cells with identical step sequence" % same)
    eq = (r.n_acc.cpu().numpy() == na) & (r.n_rej.cpu().numpy() == nr)
    _compare_h(r.h.cpu().numpy(), h, eq, "tiny")


def test_integrate_spray_full_size_sampled(spray):
    """Config at full size (262144 cells, one launch) on the GPU; a seeded
    sample of 1024 cells is recomputed by the oracle one by one. At most one
    of them (0.1%) may take another step sequence."""
    wl, mech, path, phi = spray
    S = chem.Solver(chem.Mechanism(path), device=0)
    r = S.integrate(_to(phi), wl.dt)
    torch.cuda.synchronize()
    idx = synth.sample_indices(phi.shape[0], 1024, 4)
    ref, h, na, nr, st = O.Mech(path).integrate(phi[idx], wl.dt, n_threads=NCPU)
    gst = r.status.cpu().numpy()
    assert np.array_equal(gst[idx], st)
    assert (gst == 0).all()
    _compare(phi[idx], r.phi.cpu().numpy()[idx], ref,
             (r.n_acc.cpu().numpy()[idx], r.n_rej.cpu().numpy()[idx]), (na, nr))
    eq = (r.n_acc.cpu().numpy()[idx] == na) & (r.n_rej.cpu().numpy()[idx] == nr)
    _compare_h(r.h.cpu().numpy()[idx], h, eq, "spray")
    out = r.phi.cpu().numpy()
    assert np.abs(out[:, 2:].sum(axis=1) - 1.0).max() < 1e-12


@pytest.fixture(scope="module")
def heavy(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("heavy"))
    return synth.workload_inputs("spray54_heavytail_1048576", d)


def test_spray_shear_layer_tolerances_sampled(spray):
    """The looser tolerance pair of the paper's 2-D shear-layer runs (atol
    1e-8, rtol 1e-5) on sampled cells of the full spray workload."""
    wl, mech, path, phi = spray
    S = chem.Solver(chem.Mechanism(path), chem.default_opts(schedule=chem.PERSISTENT, rtol=1e-5, atol=1e-8))
    r = S.integrate(_to(phi), wl.dt)
    torch.cuda.synchronize()
    idx = synth.sample_indices(phi.shape[0], 1024, 23)
    ref = O.Mech(path).integrate(phi[idx], wl.dt, rtol=1e-5, atol=1e-8, n_threads=NCPU)
    na, nr = r.n_acc.cpu().numpy()[idx], r.n_rej.cpu().numpy()[idx]
    assert np.array_equal(r.status.cpu().numpy()[idx], ref[4])
    _compare(phi[idx], r.phi.cpu().numpy()[idx], ref[0], (na, nr), (ref[2], ref[3]))
    # fewer substeps than at the default tolerances on the same cells
    base = O.Mech(path).integrate(phi[idx], wl.dt, n_threads=NCPU)
    assert (ref[2] + ref[3]).sum() < (base[2] + base[3]).sum()


def test_heavytail_chained_full_size_sampled(heavy):
    """1 048 576 heavy-tailed cells, ten chained steps captured in one HIP
    graph on the persistent queue with 4 waves per block and chunk 1: 256
    random cells and the 8 costliest against the oracle stepping ten times
    with the step size carried over. A cell's counters are summed over the
    ten steps; at most one sampled cell (0.1% rounded up) may differ in
    them."""
    wl, mech, path, phi = heavy
    S = chem.Solver(chem.Mechanism(path), chem.default_opts(schedule=chem.PERSISTENT, waves_per_block=4,
                                                           queue_chunk=1), device=0)
    x = _to(phi)
    h = torch.zeros(phi.shape[0], dtype=torch.float64, device=DEV)
    r = S.integrate_steps(x, wl.dt, wl.n_steps, h_io=h, out=torch.empty_like(x))
    torch.cuda.synchronize()
    gna, gnr, gst = r.n_acc.cpu().numpy(), r.n_rej.cpu().numpy(), r.status.cpu().numpy()
    assert (gst == 0).all()
    top = np.argsort(gna + gnr, kind="stable")[-8:]
    idx = np.unique(np.concatenate([synth.sample_indices(phi.shape[0], 256, 7), top]))
    M = O.Mech(path)
    cur, hh = phi[idx].copy(), np.zeros(len(idx))
    na, nr = np.zeros(len(idx), dtype=np.int64), np.zeros(len(idx), dtype=np.int64)
    for _ in range(wl.n_steps):
        cur, hh, a, b, st = M.integrate(cur, wl.dt, h_io=hh, n_threads=NCPU)
        assert (st == 0).all()
        na += a
        nr += b
    out = r.phi.cpu().numpy()
    same = _compare(phi[idx], out[idx], cur, (gna[idx], gnr[idx]), (na, nr))
    _compare_h(h.cpu().numpy()[idx], hh, (gna[idx] == na) & (gnr[idx] == nr), "heavytail")
    print("heavytail: %d/%d sampled cells with identical counts; substeps of the costliest %s"
          % (same, len(idx), (gna + gnr)[top].tolist()))
    assert np.abs(out[:, 2:].sum(axis=1) - 1.0).max() < 1e-11


def _run(S, x, dt):
    r = S.integrate(x, dt)
    torch.cuda.synchronize()
    return r


def _eq(a, b):
    return all(torch.equal(getattr(a, k), getattr(b, k)) for k in ("phi", "h", "n_acc", "n_rej", "status"))


def test_schedules_bit_identical(tiny, spray):
    for wl, mech, path, phi in (tiny, spray):
        x = _to(phi[:3000])
        S = chem.Solver(chem.Mechanism(path), device=0)
        base = _run(S, x, wl.dt)
        for kw in [dict(schedule=chem.PERSISTENT), dict(schedule=chem.PERSISTENT, queue_chunk=3),
                   dict(schedule=chem.PERSISTENT, blocks=7), dict(waves_per_block=1),
                   dict(schedule=chem.PERSISTENT, waves_per_block=2, queue_chunk=8)]:
            S.set_opts(chem.default_opts(**kw))
            assert _eq(base, _run(S, x, wl.dt)), kw
        if mech.n_species == 9:
            for cpw in (1, 4):
                S.set_opts(chem.default_opts(cells_per_wave=cpw))
                assert _eq(base, _run(S, x, wl.dt)), cpw
        # repeated run
        S.set_opts(chem.default_opts())
        assert _eq(base, _run(S, x, wl.dt))


def test_chained_steps_graph_equals_sequential(tiny):
    wl, mech, path, phi = tiny
    S = chem.Solver(chem.Mechanism(path), device=0)
    x = _to(phi)
    h = torch.zeros(x.shape[0], dtype=torch.float64, device=DEV)
    cur = x
    acc = torch.zeros(x.shape[0], dtype=torch.int32, device=DEV)
    for _ in range(3):
        r = S.integrate(cur, wl.dt, h_io=h)
        acc += r.n_acc
        cur = r.phi
    torch.cuda.synchronize()
    for sched in (chem.PLAIN, chem.PERSISTENT):
        S.set_opts(chem.default_opts(schedule=sched))
        for rep in range(2):     # second call replays the cached graph
            h2 = torch.zeros_like(h)
            out = torch.empty_like(x)
            g = S.integrate_steps(x, wl.dt, 3, h_io=h2, out=out)
            torch.cuda.synchronize()
            assert torch.equal(g.phi, cur) and torch.equal(h2, h) and torch.equal(g.n_acc, acc), (sched, rep)
    assert torch.equal(x, _to(phi))


def test_edge_cases(tiny):
    wl, mech, path, phi = tiny
    S = chem.Solver(chem.Mechanism(path), device=0)
    # empty input
    e = torch.empty((0, mech.n_species + 2), dtype=torch.float64, device=DEV)
    S.integrate(e, wl.dt)
    # ragged tail: 37 cells (not a multiple of cells per block)
    r37 = _run(S, _to(phi[:37]), wl.dt)
    r64 = _run(S, _to(phi[:64]), wl.dt)
    assert torch.equal(r37.phi, r64.phi[:37])
    # in-place
    x = _to(phi[:64])
    _ = S.integrate(x, wl.dt, out=x)
    torch.cuda.synchronize()
    assert torch.equal(x, r64.phi)
    # non-finite input and T out of range
    bad = phi[:6].copy()
    bad[0, 3] = np.nan
    bad[1, 0] = 199.0
    bad[1, 2:] = 0.0
    bad[1, 2 + mech.inert] = 1.0
    bad[3, 1] = 0.0          # pressure not positive
    bad[4, 1] = -1.0e5
    rb = _run(S, _to(bad), wl.dt)
    st = rb.status.cpu().numpy()
    assert st[0] == chem.CELL_NONFINITE and st[1] == chem.CELL_T_RANGE and st[2] == 0
    assert st[3] == chem.CELL_NONFINITE and st[4] == chem.CELL_NONFINITE and st[5] == 0
    assert np.array_equal(st, O.Mech(path).integrate(bad, wl.dt)[4])
    assert rb.phi[1, 0].item() == 199.0
    # max_steps = 1
    S.set_opts(chem.default_opts(max_steps=1))
    rm = _run(S, _to(phi[:16]), wl.dt)
    ref, h, na, nr, sto = O.Mech(path).integrate(phi[:16], wl.dt, max_steps=1)
    assert np.array_equal(rm.status.cpu().numpy(), sto)
    # bad arguments are rejected on the host
    S.set_opts(chem.default_opts())
    with pytest.raises(chem.ChemError):
        S.integrate(_to(phi[:4]), -1.0)
    y = _to(phi[:8])
    rc = chem.lib().chem_integrate(S._h, 4, 1e-6, chem.ctypes.c_void_p(y.data_ptr()),
                                   chem.ctypes.c_void_p(y[1:].data_ptr()), None, None, None, None, None)
    assert rc == -1    # partial overlap of phi_in and phi_out


def test_status_h_underflow_matches_oracle(tiny):
    """Status 2: with rtol = atol = 1e-300 every trial step is rejected (its
    error estimate is far above 1, or overflows, which also counts as a
    rejection), the substep shrinks by 0.2 and then 0.1 per attempt and falls
    below 1e-20 s. The cell keeps its input state; status, counters and the
    final substep equal the oracle's."""
    wl, mech, path, phi = tiny
    x = phi[:64]
    S = chem.Solver(chem.Mechanism(path), chem.default_opts(rtol=1e-300, atol=1e-300), device=0)
    r = _run(S, _to(x), wl.dt)
    ref, h, na, nr, st = O.Mech(path).integrate(x, wl.dt, rtol=1e-300, atol=1e-300)
    gst = r.status.cpu().numpy()
    assert (st == chem.CELL_H_UNDERFLOW).all()
    assert np.array_equal(gst, st)
    assert np.array_equal(r.n_acc.cpu().numpy(), na) and np.array_equal(r.n_rej.cpu().numpy(), nr)
    assert (na == 0).all() and (nr > 0).all()
    assert np.array_equal(r.phi.cpu().numpy(), x)
    assert np.allclose(r.h.cpu().numpy(), h, rtol=1e-12, atol=0)
    assert (h < 1e-20).all()
    # the same cells under the persistent queue
    S.set_opts(chem.default_opts(rtol=1e-300, atol=1e-300, schedule=chem.PERSISTENT))
    rp = _run(S, _to(x), wl.dt)
    assert _eq(r, rp)


def test_kernel_timing_and_workspace_info(tiny, spray):
    """Launch timing records one positive duration per integration launch made
    outside graph capture (none inside), clears on read, and stops when
    disabled; the per-wave path reports no HBM workspace."""
    wl, mech, path, phi = spray
    S = chem.Solver(chem.Mechanism(path), chem.default_opts(schedule=chem.PERSISTENT), device=0)
    assert S.workspace_info() == (0, 0)
    x = _to(phi[:2048])
    S.kernel_timing(True)
    for _ in range(3):
        S.integrate(x, wl.dt, h_io=False)
    t = S.kernel_times()
    assert len(t) == 3 and (t > 0).all() and (t < 60e3).all()
    assert len(S.kernel_times()) == 0
    out = torch.empty_like(x)
    S.integrate_steps(x, wl.dt, 2, h_io=False, out=out)       # captured: not recorded
    torch.cuda.synchronize()
    assert len(S.kernel_times()) == 0
    S.kernel_timing(False)
    S.integrate(x, wl.dt, h_io=False)
    torch.cuda.synchronize()
    assert len(S.kernel_times()) == 0
