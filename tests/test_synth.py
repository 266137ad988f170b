"""The seeded input generator: determinism, element balance, configured
counts and well-posed thermo."""
import filecmp

import numpy as np
import pytest

from paper_2112_05834_amd import synth


@pytest.mark.parametrize("name", list(synth.MECHS))
def test_mechanism_shape_and_balance(name, tmp_path):
    ns, nr, n3, nt, seed, _ = synth.MECHS[name]
    mech, path = synth.mech_cached(name, str(tmp_path / "a"))
    _, path2 = synth.mech_cached(name, str(tmp_path / "b"))
    assert filecmp.cmp(path, path2, shallow=False)          # byte-identical per seed
    assert mech.n_species == ns and mech.n_reactions == nr
    assert mech.type_counts() == (nr - n3 - nt, n3, nt)
    for r in mech.reactions:
        lhs = sum(o * mech.elem[s] for s, o in r.reac)
        rhs = sum(o * mech.elem[s] for s, o in r.prod)
        assert np.array_equal(lhs, rhs)                        # element balance, exact
        dW = sum(o * mech.W[s] for s, o in r.prod) - sum(o * mech.W[s] for s, o in r.reac)
        assert abs(dW) <= 1e-15 * max(mech.W)
        assert len({s for s, _ in r.reac}) == len(r.reac)    # species once per side
    used = {s for r in mech.reactions for s, _ in r.reac + r.prod}
    assert used == set(range(ns - 1))                          # every non-inert species reacts
    assert mech.inert not in used


@pytest.mark.parametrize("name", list(synth.MECHS))
def test_heat_capacity_positive_monotone(name, tmp_path):
    mech, _ = synth.mech_cached(name, str(tmp_path))
    T = np.linspace(200.0, 6000.0, 2001)
    for a in mech.nasa_lo:
        cp = a[0] + a[1] * T + a[2] * T ** 2 + a[3] * T ** 3 + a[4] * T ** 4
        assert np.all(cp > 0)
        assert np.all(np.diff(cp) >= -1e-12)


@pytest.mark.parametrize("wl", list(synth.WORKLOADS))
def test_states(wl, tmp_path):
    w = synth.WORKLOADS[wl]
    n = min(4096, w.n_cells)
    wl_, mech, path, phi = synth.workload_inputs(wl, str(tmp_path), n_cells=n)
    _, _, _, phi2 = synth.workload_inputs(wl, str(tmp_path), n_cells=n)
    assert np.array_equal(phi, phi2)
    assert phi.shape == (n, mech.n_species + 2) and phi.flags.c_contiguous
    assert np.all(phi[:, 1] == w.pressure)
    assert np.all(phi[:, 2:] >= 0)
    assert np.allclose(phi[:, 2:].sum(axis=1), 1.0, atol=1e-14)
    assert phi[:, 0].min() > 300 and phi[:, 0].max() < 3500


def test_sample_indices():
    a = synth.sample_indices(262144, 4096, 3)
    assert len(a) == 4096 and len(set(a.tolist())) == 4096 and np.all(np.diff(a) > 0)
    assert np.array_equal(a, synth.sample_indices(262144, 4096, 3))
