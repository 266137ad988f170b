"""GPU parity of the method's variants through the C ABI, against the oracle
run with the same variant:

- ROS4 (Shampine's order-4(3) Rosenbrock scheme) as a table swap for Rodas3,
  on the per-wave kernel (9 and 54 species) and the workgroup kernel (160);
- the forward-difference Jacobian (the conventional finite-difference
  Jacobian the paper replaces with an analytical one) on the same kernels.

Tolerances and the step-sequence allowance are those of the Rodas3 parity
tests: T relative 1e-8 and Y within 1e-10 + 1e-6 |Y| on cells with the
oracle's accepted/rejected counts; at most 0.1% of cells (at least one) on
another sequence, those within ten times the tolerance. A forward-difference
column divides a difference of two right-hand sides by an increment of
~1e-8 relative, so the last-bit differences between the GPU's and the
oracle's right-hand sides reach the FD Jacobians at ~1e-8 relative; the
integrations still meet the same bar.
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


def _compare(phi0, gpu, ref, counts_gpu, counts_ref, what):
    na, nr = counts_gpu
    ona, onr = counts_ref
    same = (na == ona) & (nr == onr)
    n = len(same)
    assert (~same).sum() <= max(1, n // 1000), "%s: %d of %d cells on another step sequence" % (what, (~same).sum(), n)
    dT = np.abs(gpu[:, 0] - ref[:, 0])
    dY = np.abs(gpu[:, 2:] - ref[:, 2:])
    tolY = 1e-10 + 1e-6 * np.abs(ref[:, 2:])
    assert not (same & (dT > 1e-8 * np.abs(ref[:, 0]))).any(), what
    assert not (same[:, None] & (dY > tolY)).any(), what
    if (~same).any():
        assert np.all(dT[~same] <= 10 * 1e-6 * np.abs(ref[~same, 0])), what
        assert np.all(dY[~same] <= 10 * tolY[~same]), what
    assert np.array_equal(gpu[:, 1], phi0[:, 1])
    print("%s: %d/%d cells on the oracle's step sequence, max |dT|/T %.2e" % (what, same.sum(), n, (dT / ref[:, 0]).max()),
          flush=True)


CASES = [("tiny9_1024", 1024, None), ("spray54_262144", 262144, 256), ("large160_524288", 48, None)]


VARIANTS = {
    "ros4": (dict(scheme=chem.ROS4), dict(scheme=O.ROS4)),
    "fd": (dict(jacobian=chem.JAC_FD), dict(jacobian=O.JAC_FD)),
    "nobath": (dict(state=chem.STATE_NO_BATH), dict(state=O.STATE_NO_BATH)),
    "ros4_fd_nobath": (dict(scheme=chem.ROS4, jacobian=chem.JAC_FD, state=chem.STATE_NO_BATH),
                       dict(scheme=O.ROS4, jacobian=O.JAC_FD, state=O.STATE_NO_BATH)),
}


@pytest.mark.parametrize("name,n_gpu,n_check", CASES)
@pytest.mark.parametrize("variant", ["ros4", "fd", "nobath", "ros4_fd_nobath"])
def test_variant_matches_oracle(tmp_path, name, n_gpu, n_check, variant):
    """ros4: Shampine's scheme; fd: forward-difference Jacobian; nobath: the
    last species (the bath gas) not integrated, its mass fraction 1 - the
    sum of the others (n = Ns); and the three together."""
    wl, mech, path, phi = synth.workload_inputs(name, str(tmp_path), n_cells=n_gpu)
    kw, okw = VARIANTS[variant]
    if "fd" in variant and name == "spray54_262144":
        n_check = 128
    S = chem.Solver(chem.Mechanism(path), chem.default_opts(schedule=chem.PERSISTENT, **kw), device=0)
    r = S.integrate(_to(phi), wl.dt)
    torch.cuda.synchronize()
    idx = np.arange(phi.shape[0]) if n_check is None else synth.sample_indices(phi.shape[0], n_check, 29)
    ref, h, na, nr, st = O.Mech(path).integrate(phi[idx], wl.dt, n_threads=NCPU, **okw)
    gst = r.status.cpu().numpy()[idx]
    assert np.array_equal(gst, st)
    _compare(phi[idx], r.phi.cpu().numpy()[idx], ref, (r.n_acc.cpu().numpy()[idx], r.n_rej.cpu().numpy()[idx]),
             (na, nr), "%s %s" % (variant, name))
    if "nobath" in variant:
        out = r.phi.cpu().numpy()
        assert np.abs(out[:, 2:].sum(axis=1) - 1.0).max() <= 1e-15
    # plain and persistent schedules give the same bits for the variant too
    if name != "spray54_262144":
        S.set_opts(chem.default_opts(schedule=chem.PLAIN, **kw))
        r2 = S.integrate(_to(phi), wl.dt)
        torch.cuda.synchronize()
        for k in ("phi", "h", "n_acc", "n_rej", "status"):
            assert torch.equal(getattr(r, k), getattr(r2, k)), k


def test_rodas3_default_unchanged_by_variant_options(tmp_path):
    """Options left at their defaults select Rodas3 with the analytical
    Jacobian: the same bits as a solver created without them."""
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", str(tmp_path), n_cells=256)
    S = chem.Solver(chem.Mechanism(path), device=0)
    a = S.integrate(_to(phi), wl.dt)
    S.set_opts(chem.default_opts(scheme=chem.RODAS3, jacobian=chem.JAC_ANALYTICAL))
    b = S.integrate(_to(phi), wl.dt)
    torch.cuda.synchronize()
    assert torch.equal(a.phi, b.phi) and torch.equal(a.n_acc, b.n_acc)
    with pytest.raises(chem.ChemError):
        S.set_opts(chem.default_opts(scheme=5))
    with pytest.raises(chem.ChemError):
        S.set_opts(chem.default_opts(jacobian=2))


@pytest.mark.parametrize("name", ["tiny9_1024", "spray54_262144"])
def test_rocsolver_lu_matches_wave_lu(tmp_path, name):
    """rocSOLVER's batched getrf/getrs on the transposes (column-major) of the
    matrices the library's LU factors row-major: identical pivots (LAPACK's
    first-maximum rule on both sides; rocSOLVER's are 1-based), factors within
    1e-12 of the largest entry, solutions within 1e-10."""
    wl, mech, path, phi = synth.workload_inputs(name, str(tmp_path), n_cells=64)
    S = chem.Solver(chem.Mechanism(path), device=0)
    n = mech.n_species + 1
    M = O.Mech(path)
    rng = np.random.Generator(np.random.PCG64(n))
    A = rng.normal(size=(48, n, n)) + 3.0 * np.eye(n)[None]
    for c in range(16):
        y = np.concatenate([[phi[c, 0]], phi[c, 2:]])
        A[c] = np.eye(n) / (0.5 * 1e-8) - M.jac(phi[c, 1], y)
    b = rng.normal(size=(48, n))
    Ag, piv, info, bg = S.lu_batch(_to(A), _to(b))
    # column-major copies for the library: element (i, j) of matrix k at [k, j, i]
    Ar, pivr, infor, br = chem.lu_batch_rocsolver(_to(A).transpose(1, 2).contiguous(), _to(b))
    torch.cuda.synchronize()
    assert (info.cpu() == 0).all() and (infor.cpu() == 0).all()
    assert torch.equal(piv.cpu() + 1, pivr.cpu())
    F, Fr = Ag.cpu().numpy(), Ar.transpose(1, 2).cpu().numpy()
    for k in range(A.shape[0]):
        assert np.max(np.abs(F[k] - Fr[k])) <= 1e-12 * np.max(np.abs(A[k])), k
    assert np.max(np.abs(bg.cpu().numpy() - br.cpu().numpy())) <= 1e-10 * np.max(np.abs(bg.cpu().numpy()))
