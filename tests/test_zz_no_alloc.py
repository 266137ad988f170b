"""The allocation-free entry point (chem_integrate_noalloc) through the C ABI
against chem_integrate on the same inputs: results equal in every bit (same
kernels, same per-cell arithmetic under any schedule), on two calls in a row,
the second with fewer cells, for the per-wave kernel (54 species: the queue
head in the static scratch) and the workgroup kernel (160 species: the J and
M workspace slots in the static scratch as well)."""
import numpy as np
import pytest
import torch

from paper_2112_05834_amd import chem, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _same(a, b):
    return all(torch.equal(getattr(a, k), getattr(b, k)) for k in ("phi", "h", "n_acc", "n_rej", "status"))


@pytest.mark.parametrize("workload,sizes", [("spray54_262144", (4096, 1000)), ("large160_524288", (600, 97))])
def test_noalloc_equals_integrate_two_calls(tmp_path, workload, sizes):
    wl, mech, path, phi = synth.workload_inputs(workload, str(tmp_path), n_cells=max(sizes))
    S = chem.Solver(chem.Mechanism(path), chem.default_opts(schedule=chem.PERSISTENT), device=0)
    for n in sizes:
        print("noalloc: %s, %d cells" % (workload, n), flush=True)
        x = torch.from_numpy(np.ascontiguousarray(phi[:n])).to(DEV)
        h0 = torch.zeros(n, dtype=torch.float64, device=DEV)
        ref = S.integrate(x, wl.dt, h_io=h0.clone())
        got = S.integrate_noalloc(x, wl.dt, h_io=h0.clone())
        torch.cuda.synchronize()
        assert _same(ref, got), (workload, n)
        assert (got.status == 0).all()
    # in place, as chem_integrate allows
    y = torch.from_numpy(np.ascontiguousarray(phi[:sizes[1]])).to(DEV)
    ref = S.integrate(y, wl.dt, h_io=False)
    S.integrate_noalloc(y, wl.dt, h_io=False, out=y)
    torch.cuda.synchronize()
    assert torch.equal(ref.phi, y)


def test_noalloc_rejects_bad_arguments(tmp_path):
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", str(tmp_path), n_cells=8)
    S = chem.Solver(chem.Mechanism(path), device=0)
    x = torch.from_numpy(phi).to(DEV)
    with pytest.raises(chem.ChemError) as e:
        S.integrate_noalloc(x, -1.0)
    assert e.value.code == -1
    e = torch.empty((0, mech.n_species + 2), dtype=torch.float64, device=DEV)
    S.integrate_noalloc(e, wl.dt)
