"""Zonal reference mapping on the GPU (paper: Methodology, the DLBFoam
paragraph) through the C ABI, against the oracle's reading of it.

- Z: identical bits to the oracle (same sums in the same order, one fused
  multiply-add per term on both sides), so the zone and mapping decisions are
  compared exactly;
- integrated cells: the parity bar of the plain integration (T relative
  1e-8, Y 1e-10 + 1e-6 |Y| on cells with equal step counts), and identical
  bits to chem_integrate on the GPU, whose per-cell results do not depend on
  the schedule;
- mapped cells: exactly phi_in + (reference out - reference in), recomputed
  on the host from the GPU's own outputs.
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
Z_MAX, T_TOL = 1e-6, 1.0


def _to(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _states(mech_name, n, d, pressure=6.0e6, seed=106):
    mech, path = synth.mech_cached(mech_name, d)
    return mech, path, synth.generate_states(mech, n, pressure, "ambient", seed)


def _solver(path, mech, z_max=Z_MAX, t_tol=T_TOL, dz=0.0, **kw):
    S = chem.Solver(chem.Mechanism(path), chem.default_opts(schedule=chem.PERSISTENT, **kw))
    c, yf, yo = synth.bilger_streams(mech)
    S.zone_config(c, yf, yo, z_max, t_tol, dz=dz)
    return S


def _rule_bands(z, T, z_max, t_tol, dz):
    """The banded mapping rule written out on the host from the oracle's Z:
    (band + 1 of mapped cells else 0, reference cell of each zone cell)."""
    n = len(z)
    zone = np.nonzero(z <= z_max)[0]
    band = np.floor(np.maximum(z[zone], 0.0) / dz).astype(np.int64) if dz > 0 else np.zeros(len(zone), np.int64)
    _, first = np.unique(band, return_index=True)          # first occurrence in index order
    refcell = dict(zip(band[first], zone[first]))
    ref = np.array([refcell[b] for b in band], dtype=np.int64)
    mapped = np.zeros(n, dtype=np.int8)
    hit = (zone != ref) & (np.abs(T[zone] - T[ref]) <= t_tol)
    mapped[zone[hit]] = band[hit] + 1
    refs = np.full(n, -1, dtype=np.int64)
    refs[zone] = ref
    return mapped, refs


def _np(r):
    return (r.phi.cpu().numpy(), r.h.cpu().numpy(), r.n_acc.cpu().numpy(), r.n_rej.cpu().numpy(),
            r.status.cpu().numpy())


def _rule(z, T, z_max, t_tol):
    """The mapping rule written out on the host from the oracle's Z."""
    zone = np.nonzero(z <= z_max)[0]
    mapped = np.zeros(len(z), dtype=bool)
    if zone.size:
        ref = zone[0]
        mapped[zone] = np.abs(T[zone] - T[ref]) <= t_tol
        mapped[ref] = False
        return mapped, int(ref)
    return mapped, -1


def _check_mapped(phi0, out, mapped, ref, na, nr, st):
    m = np.nonzero(mapped)[0]
    if not m.size:
        return
    want = phi0[m].copy()
    want[:, 0] = phi0[m, 0] + (out[ref, 0] - phi0[ref, 0])
    want[:, 2:] = phi0[m, 2:] + (out[ref, 2:] - phi0[ref, 2:])
    assert np.array_equal(out[m], want)
    assert (na[m] == 0).all() and (nr[m] == 0).all() and (st[m] == st[ref]).all()


def _compare_integrated(gpu, ref, same):
    dT = np.abs(gpu[:, 0] - ref[:, 0])
    dY = np.abs(gpu[:, 2:] - ref[:, 2:])
    tolY = 1e-10 + 1e-6 * np.abs(ref[:, 2:])
    assert (~same).sum() <= max(1, len(same) // 1000)
    assert not (same & (dT > 1e-8 * np.abs(ref[:, 0]))).any()
    assert not (same[:, None] & (dY > tolY)).any()
    assert np.all(dT[~same] <= 1e-5 * np.abs(ref[~same, 0]))


@pytest.mark.parametrize("mech_name", ["tiny9", "spray54", "large160"])
def test_mixture_fraction_identical_to_oracle(tmp_path, mech_name):
    mech, path, phi = _states(mech_name, 4099, str(tmp_path))
    S = _solver(path, mech)
    z = S.mixture_fraction(_to(phi)).cpu().numpy()
    c, yf, yo = synth.bilger_streams(mech)
    zo = O.Mech(path).mixture_fraction(c, yf, yo, phi)
    assert np.array_equal(z, zo)
    assert 0.5 < (zo <= Z_MAX).mean() < 0.7          # the ambient share of the recipe


@pytest.mark.parametrize("mech_name,n", [("tiny9", 640), ("spray54", 193), ("large160", 20)])
def test_zonal_against_oracle(tmp_path, mech_name, n):
    print("zonal parity", mech_name, n, flush=True)
    mech, path, phi = _states(mech_name, n, str(tmp_path))
    dt = 5e-7 if mech_name == "large160" else 1e-6
    S = _solver(path, mech)
    r, m = S.integrate_zonal(_to(phi), dt)
    torch.cuda.synchronize()
    out, h, na, nr, st = _np(r)
    mapped = m.cpu().numpy().astype(bool)
    c, yf, yo = synth.bilger_streams(mech)
    o_out, o_h, o_na, o_nr, o_st, o_mapped = O.Mech(path).integrate_zonal(
        phi, dt, c, yf, yo, Z_MAX, T_TOL, n_threads=NCPU)
    assert np.array_equal(mapped, o_mapped)
    assert mapped.sum() >= n // 3 and (~mapped).sum() >= 2
    assert np.array_equal(st, o_st)
    solved = ~mapped
    same = (na[solved] == o_na[solved]) & (nr[solved] == o_nr[solved])
    _compare_integrated(out[solved], o_out[solved], same)
    assert np.array_equal(out[:, 1], phi[:, 1])
    ref = int(np.nonzero(O.Mech(path).mixture_fraction(c, yf, yo, phi) <= Z_MAX)[0][0])
    _check_mapped(phi, out, mapped, ref, na, nr, st)


def test_zonal_bands_against_oracle(tmp_path):
    """Z bands (dz = 0.01 up to z_max = 0.3): the unburnt and hot cells of
    the spray recipe fall into 31 bands, each mapped from its own reference."""
    mech, path, phi = _states("spray54", 400, str(tmp_path))
    S = _solver(path, mech, z_max=0.3, t_tol=5.0, dz=0.01)
    r, m = S.integrate_zonal(_to(phi), 1e-6)
    out, h, na, nr, st = _np(r)
    mapped = m.cpu().numpy()
    c, yf, yo = synth.bilger_streams(mech)
    o_out, o_h, o_na, o_nr, o_st, o_mapped = O.Mech(path).integrate_zonal(
        phi, 1e-6, c, yf, yo, 0.3, 5.0, dz=0.01, n_threads=NCPU)
    assert np.array_equal(mapped, o_mapped)
    assert len(np.unique(mapped[mapped > 0])) >= 3          # several bands map cells
    assert np.array_equal(st, o_st)
    solved = mapped == 0
    same = (na[solved] == o_na[solved]) & (nr[solved] == o_nr[solved])
    _compare_integrated(out[solved], o_out[solved], same)
    z = O.Mech(path).mixture_fraction(c, yf, yo, phi)
    want, refs = _rule_bands(z, phi[:, 0], 0.3, 5.0, 0.01)
    assert np.array_equal(mapped, want)
    for i in np.nonzero(mapped)[0]:
        ref = refs[i]
        assert np.array_equal(out[i, 2:], phi[i, 2:] + (out[ref, 2:] - phi[ref, 2:]))
        assert out[i, 0] == phi[i, 0] + (out[ref, 0] - phi[ref, 0])
        assert na[i] == 0 and st[i] == st[ref]


def test_zonal_bands_full_size_headline_cells(tmp_path):
    """The headline spray cells (262 144) with 60 Z bands up to z_max = 0.3:
    flags as the host rule on the oracle's Z, integrated cells identical to
    chem_integrate, mapped cells their band reference's change exactly."""
    wl, mech, path, phi = synth.workload_inputs("spray54_262144", str(tmp_path))
    S = _solver(path, mech, z_max=0.3, t_tol=2.0, dz=0.005)
    x = _to(phi)
    r, m = S.integrate_zonal(x, wl.dt)
    rz = _np(r)
    mapped = m.cpu().numpy()
    rp = _np(S.integrate(x, wl.dt))
    c, yf, yo = synth.bilger_streams(mech)
    z = O.Mech(path).mixture_fraction(c, yf, yo, phi)
    want, refs = _rule_bands(z, phi[:, 0], 0.3, 2.0, 0.005)
    assert np.array_equal(mapped, want)
    solved = mapped == 0
    for a, b in zip(rz, rp):
        assert np.array_equal(a[solved], b[solved])
    out = rz[0]
    idx = np.nonzero(mapped)[0]
    rr = refs[idx]
    assert np.array_equal(out[idx, 2:], phi[idx, 2:] + (out[rr, 2:] - phi[rr, 2:]))
    assert np.array_equal(out[idx, 0], phi[idx, 0] + (out[rr, 0] - phi[rr, 0]))
    dT = np.abs(out[idx, 0] - rp[0][idx, 0])
    print("bands: %.1f%% mapped in %d bands, max |T_mapped - T_integrated| = %.3e K"
          % (100 * (mapped > 0).mean(), len(np.unique(mapped[mapped > 0])), dT.max()), flush=True)


def test_zone_boundary_is_decided_in_the_same_bits(tmp_path):
    """z_max set to one cell's Z exactly (as the oracle computes it) puts that
    cell in the zone; the next double below takes it out. Only a Z with the
    oracle's bits gets both right."""
    mech, path, phi = _states("spray54", 1000, str(tmp_path))
    c, yf, yo = synth.bilger_streams(mech)
    z = O.Mech(path).mixture_fraction(c, yf, yo, phi)
    # k: a fuel-bearing cell of median Z, unique to it; the reference stays the
    # first ambient cell, and t_tol = 1e4 K maps every other zone cell
    rest = np.nonzero(z > Z_MAX)[0]
    k = int(rest[np.argsort(z[rest])[len(rest) // 2]])
    assert (z == z[k]).sum() == 1 and k > np.nonzero(z <= Z_MAX)[0][0]
    x = _to(phi)
    for zm, inside in ((z[k], True), (np.nextafter(z[k], -np.inf), False)):
        S = _solver(path, mech, z_max=float(zm), t_tol=1e4)
        _, m = S.integrate_zonal(x, 1e-6)
        mapped = m.cpu().numpy().astype(bool)
        want, _ = _rule(z, phi[:, 0], zm, 1e4)
        assert np.array_equal(mapped, want)
        assert mapped[k] == inside


def test_zonal_full_size_workload(tmp_path):
    """The ambient spray workload at full size (262 144 cells) in the launch
    configuration of the benchmark."""
    wl, mech, path, phi = synth.workload_inputs("spray54_ambient_262144", str(tmp_path))
    n = phi.shape[0]
    print("zonal full size", n, flush=True)
    S = _solver(path, mech)
    x = _to(phi)
    r, m = S.integrate_zonal(x, wl.dt)
    rz = _np(r)
    mapped = m.cpu().numpy().astype(bool)
    rp = _np(S.integrate(x, wl.dt))
    c, yf, yo = synth.bilger_streams(mech)
    M = O.Mech(path)
    z = M.mixture_fraction(c, yf, yo, phi)
    want, ref = _rule(z, phi[:, 0], Z_MAX, T_TOL)
    assert np.array_equal(mapped, want)
    assert 0.55 < mapped.mean() < 0.65
    solved = ~mapped
    for a, b in zip(rz, rp):
        assert np.array_equal(a[solved], b[solved])
    out, h, na, nr, st = rz
    _check_mapped(phi, out, mapped, ref, na, nr, st)
    # sampled integrated cells against the oracle
    idx = np.nonzero(solved)[0][synth.sample_indices(int(solved.sum()), 32, 11)]
    o = M.integrate(phi[idx], wl.dt, n_threads=NCPU)
    _compare_integrated(out[idx], o[0], (na[idx] == o[2]) & (nr[idx] == o[3]))
    # Z is a conserved scalar: the integrated cells keep theirs
    z_out = S.mixture_fraction(r.phi).cpu().numpy()
    assert np.abs(z_out[solved] - z[solved]).max() < 1e-12
    # what the mapping changes against integrating every cell
    dT = np.abs(out[mapped, 0] - rp[0][mapped, 0])
    print("mapped %.1f%%, max |T_mapped - T_integrated| = %.3e K" % (100 * mapped.mean(), dT.max()), flush=True)
    assert dT.max() <= T_TOL


def test_zonal_in_place_and_reuse(tmp_path):
    mech, path, phi = _states("spray54", 4096, str(tmp_path))
    S = _solver(path, mech)
    r1, m1 = S.integrate_zonal(_to(phi), 1e-6)
    a = _np(r1)
    x = _to(phi)
    r2, m2 = S.integrate_zonal(x, 1e-6, out=x)
    b = _np(r2)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert torch.equal(m1, m2)
    # a smaller call reuses the buffers; its zone has its own reference
    r3, m3 = S.integrate_zonal(_to(phi[1000:3000]), 1e-6)
    c = _np(r3)
    Sb = _solver(path, mech)
    r4, m4 = Sb.integrate_zonal(_to(phi[1000:3000]), 1e-6)
    for u, v in zip(c, _np(r4)):
        assert np.array_equal(u, v)
    assert torch.equal(m3, m4)


def test_zonal_degenerate_cases(tmp_path):
    mech, path, phi = _states("spray54", 2048, str(tmp_path))
    x = _to(phi)
    # no zone: identical to the plain integration
    S = _solver(path, mech, z_max=-1.0)
    r, m = S.integrate_zonal(x, 1e-6)
    assert int(m.sum()) == 0
    for u, v in zip(_np(r), _np(S.integrate(x, 1e-6))):
        assert np.array_equal(u, v)
    # t_tol = 0: only cells at exactly the reference temperature are mapped
    S0 = _solver(path, mech, t_tol=0.0)
    _, m0 = S0.integrate_zonal(x, 1e-6)
    assert int(m0.sum()) == 0
    # empty input
    r_e, m_e = S0.integrate_zonal(x[:0], 1e-6)
    assert r_e.phi.shape[0] == 0 and m_e.numel() == 0
    # every cell in the zone and within t_tol: all take cell 0's change and its
    # status; cell 0 is inert gas below the thermo range, so it stops at once
    phi = phi.copy()
    phi[0, 0] = 199.0
    phi[0, 2:] = 0.0
    phi[0, 2 + mech.inert] = 1.0
    Sa = _solver(path, mech, z_max=2.0, t_tol=1e4)
    ra, ma = Sa.integrate_zonal(_to(phi), 1e-6)
    out, h, na, nr, st = _np(ra)
    mapped = ma.cpu().numpy().astype(bool)
    assert not mapped[0] and mapped[1:].all()
    assert st[0] == chem.CELL_T_RANGE and out[0, 0] == 199.0
    _check_mapped(phi, out, mapped, 0, na, nr, st)
    assert np.array_equal(out[1:], phi[1:])


def test_zonal_null_mapped_and_cells_per_wave(tmp_path):
    """Through the C ABI with mapped = NULL (the solver's own flag buffer),
    and with 1 and 4 cells per wave of the 10-component kernel: the same
    bits every time."""
    import ctypes
    mech, path, phi = _states("tiny9", 777, str(tmp_path))
    x = _to(phi)
    outs = []
    for cpw in (1, 4):
        S = _solver(path, mech, cells_per_wave=cpw)
        r, m = S.integrate_zonal(x, 1e-6)
        outs.append((_np(r), m.cpu().numpy()))
        o = torch.empty_like(x)
        na = torch.empty(777, dtype=torch.int32, device=DEV)
        nr = torch.empty_like(na)
        st = torch.empty(777, dtype=torch.int8, device=DEV)
        h = torch.zeros(777, dtype=torch.float64, device=DEV)
        vp = ctypes.c_void_p
        rc = chem.lib().chem_integrate_zonal(S._h, 777, 1e-6, vp(x.data_ptr()), vp(o.data_ptr()), vp(h.data_ptr()),
                                             vp(na.data_ptr()), vp(nr.data_ptr()), vp(st.data_ptr()), None,
                                             vp(torch.cuda.current_stream().cuda_stream))
        assert rc == 0
        torch.cuda.synchronize()
        for u, v in zip(_np(r), (o.cpu().numpy(), h.cpu().numpy(), na.cpu().numpy(), nr.cpu().numpy(),
                                 st.cpu().numpy())):
            assert np.array_equal(u, v)
    for u, v in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(u, v)
    assert np.array_equal(outs[0][1], outs[1][1]) and outs[0][1].sum() > 300


def test_zonal_and_chained_steps_captured_by_the_caller(tmp_path):
    """A caller's own graph capture (torch.cuda.graph) of a zonal call and of
    chained steps, after one eager call of each has allocated the solver's
    buffers: every replay, with eager work and synchronisation between the
    replays, gives the eager call's bits."""
    mech, path, phi = _states("spray54", 2048, str(tmp_path))
    S = _solver(path, mech)
    x = _to(phi)
    out_z = torch.empty_like(x)
    out_c = torch.empty_like(x)
    rz, mz = S.integrate_zonal(x, 1e-6, h_io=False, out=out_z)
    rc = S.integrate_steps(x, 1e-6, 3, h_io=False, out=out_c)
    torch.cuda.synchronize()
    want = [t.clone() for t in (rz.phi, rz.n_acc, rz.n_rej, rz.status, mz, rc.phi, rc.n_acc, rc.n_rej, rc.status)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gz, gm = S.integrate_zonal(x, 1e-6, h_io=False, out=out_z)
        gc = S.integrate_steps(x, 1e-6, 3, h_io=False, out=out_c)
    for rep in range(3):
        out_z.fill_(-1.0)
        out_c.fill_(-1.0)
        junk = (x * 2.0).sum()                     # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (gz.phi, gz.n_acc, gz.n_rej, gz.status, gm, gc.phi, gc.n_acc, gc.n_rej, gc.status)
        for a, b in zip(got, want):
            assert torch.equal(a, b), "replay %d differs" % rep
        assert torch.isfinite(junk)


def test_zone_config_errors(tmp_path):
    mech, path, phi = _states("tiny9", 4, str(tmp_path))
    S = chem.Solver(chem.Mechanism(path), chem.default_opts())
    x = torch.from_numpy(phi).to(DEV)
    with pytest.raises(chem.ChemError) as e:
        S.integrate_zonal(x, 1e-6)
    assert e.value.code == -5
    c, yf, yo = synth.bilger_streams(mech)
    S.zone_config(c, yf, yo, Z_MAX, T_TOL)
    with pytest.raises(chem.ChemError):
        S.zone_config(c, yo, yo, Z_MAX, T_TOL)
    # a failed configuration leaves no zone definition behind
    with pytest.raises(chem.ChemError) as e:
        S.integrate_zonal(x, 1e-6)
    assert e.value.code == -5
    with pytest.raises(chem.ChemError):
        S.zone_config(c, yf, yo, Z_MAX, -1.0)
    with pytest.raises(chem.ChemError):
        S.zone_config(c, yf, yo, float("nan"), T_TOL)
    # bands: a negative width, and more than 64 bands for z_max
    # a rejected band width leaves no zone behind either, even though the
    # zone itself was configured before the width was checked
    for bad_dz in (-0.01, 0.001, float("inf")):
        S.zone_config(c, yf, yo, Z_MAX, T_TOL)
        S.integrate_zonal(x, 1e-6)
        with pytest.raises(chem.ChemError):
            S.zone_config(c, yf, yo, 0.3, T_TOL, dz=bad_dz)
        with pytest.raises(chem.ChemError) as e:
            S.integrate_zonal(x, 1e-6)
        assert e.value.code == -5, bad_dz
