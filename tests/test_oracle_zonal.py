"""Pins of the oracle's mixture fraction and zonal reference mapping (paper:
Methodology, the DLBFoam paragraph; Bilger's mixture fraction), on the CPU.

- closed forms: Z = 1 in the fuel stream, 0 in the oxidiser stream, linear in
  between;
- a textbook case: methane in air, where Bilger's coupling vanishes at
  stoichiometry, so Z of the stoichiometric mixture is 1/(1 + s/Y_O2) with
  s = 2 W_O2 / W_CH4 (about 0.055), the fully burnt products of that
  mixture have the same Z (element conservation), and so do pure CO2 and
  pure H2O;
- an invariant: element-balanced reactions leave Z unchanged, so the
  oracle's integration must conserve it;
- the mapping rule on tiny hand-built inputs.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2112_05834_amd import synth

W = {"H": 1.008e-3, "C": 12.011e-3, "O": 15.999e-3, "N": 14.007e-3}
SPECIES = {  # atoms of H, C, O, N
    "CH4": (4, 1, 0, 0), "O2": (0, 0, 2, 0), "N2": (0, 0, 0, 2), "CO2": (0, 1, 2, 0), "H2O": (2, 0, 1, 0),
}


def _methane_air(tmp_path):
    lines = ["chemmech 1", "elements 4"] + ["%s %r" % (e, w) for e, w in W.items()]
    lines.append("species %d" % len(SPECIES))
    nasa = "3.5 0 0 0 0 -1000 4"
    for name, a in SPECIES.items():
        wi = sum(k * w for k, w in zip(a, W.values()))
        lines += ["%s %r 200 1000 6000 %s" % (name, wi, " ".join(map(str, a))), nasa, nasa]
    lines += ["reactions 0", "end"]
    p = tmp_path / "ch4air.mech"
    p.write_text("\n".join(lines) + "\n")
    Wsp = {n: sum(k * w for k, w in zip(a, W.values())) for n, a in SPECIES.items()}
    return O.Mech(str(p)), list(SPECIES), Wsp


def _phi(Y, T=300.0, p=101325.0):
    Y = np.atleast_2d(np.asarray(Y, dtype=np.float64))
    out = np.zeros((Y.shape[0], Y.shape[1] + 2))
    out[:, 0], out[:, 1], out[:, 2:] = T, p, Y
    return out


COUPLING = np.array([0.5, 2.0, -1.0, 0.0])   # H, C, O, N


def test_element_counts_round_trip(tmp_path):
    M, names, _ = _methane_air(tmp_path)
    assert (M.elements() == np.array([SPECIES[n] for n in names])).all()


def test_streams_are_zero_and_one_and_z_is_linear(tmp_path):
    M, names, _ = _methane_air(tmp_path)
    yf = np.array([1.0, 0, 0, 0, 0])
    yo = np.array([0, 0.233, 0.767, 0, 0])
    z = M.mixture_fraction(COUPLING, yf, yo, _phi([yf, yo]))
    assert z[0] == 1.0 and z[1] == 0.0
    f = np.random.default_rng(3).uniform(0, 1, 50)
    mix = f[:, None] * yf + (1 - f[:, None]) * yo
    assert np.allclose(M.mixture_fraction(COUPLING, yf, yo, _phi(mix)), f, rtol=0, atol=1e-14)


def test_methane_air_stoichiometric_mixture_fraction(tmp_path):
    M, names, Wsp = _methane_air(tmp_path)
    yf = np.array([1.0, 0, 0, 0, 0])
    yo = np.array([0, 0.233, 0.767, 0, 0])
    s = 2 * Wsp["O2"] / Wsp["CH4"]
    z_st = 1.0 / (1.0 + s / 0.233)
    assert abs(z_st - 0.055) < 1e-3                      # the textbook value
    unburnt = z_st * yf + (1 - z_st) * yo
    n = z_st / Wsp["CH4"]                                # mol CH4 per kg, burnt to CO2 + 2 H2O
    burnt = np.array([0.0, 0.0, (1 - z_st) * 0.767, n * Wsp["CO2"], 2 * n * Wsp["H2O"]])
    assert abs(burnt.sum() - 1.0) < 1e-12
    z = M.mixture_fraction(COUPLING, yf, yo, _phi([unburnt, burnt]))
    assert abs(z[0] - z_st) < 1e-12 and abs(z[1] - z_st) < 1e-12
    # Bilger's weights vanish on the fully oxidised products themselves, so pure
    # CO2 and pure H2O sit at stoichiometry too; a wrong weight moves them off
    pure = _phi([[0, 0, 0, 1.0, 0], [0, 0, 0, 0, 1.0]])
    assert np.abs(M.mixture_fraction(COUPLING, yf, yo, pure) - z_st).max() < 1e-12
    for bad in ([0.5, 2.0, 1.0, 0.0], [1.0, 2.0, -1.0, 0.0], [0.5, 1.0, -1.0, 0.0]):
        assert np.abs(M.mixture_fraction(np.array(bad), yf, yo, pure) - z_st).max() > 1e-3


def test_equal_streams_are_an_error(tmp_path):
    M, _, _ = _methane_air(tmp_path)
    y = np.array([0, 0.233, 0.767, 0, 0])
    with pytest.raises(ValueError):
        M.mixture_fraction(COUPLING, y, y, _phi([y]))


@pytest.mark.parametrize("name,n", [("tiny9_1024", 48), ("spray54_262144", 32)])
def test_integration_conserves_mixture_fraction(tmp_path, name, n):
    wl, mech, path, phi = synth.workload_inputs(name, str(tmp_path), n_cells=n)
    M = O.Mech(path)
    c, yf, yo = synth.bilger_streams(mech)
    out = M.integrate(phi, wl.dt)[0]
    assert np.abs(out[:, 0] - phi[:, 0]).max() > 10.0      # the chemistry did something
    z0 = M.mixture_fraction(c, yf, yo, phi)
    z1 = M.mixture_fraction(c, yf, yo, out)
    assert np.abs(z1 - z0).max() < 1e-13


def _zonal_case(tmp_path):
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", str(tmp_path), n_cells=12)
    M = O.Mech(path)
    c, yf, yo = synth.bilger_streams(mech)
    return wl, M, c, yf, yo, phi.copy()


def test_zonal_without_zone_is_plain_integration(tmp_path):
    wl, M, c, yf, yo, phi = _zonal_case(tmp_path)
    out, h, na, nr, st, mapped = M.integrate_zonal(phi, wl.dt, c, yf, yo, z_max=-1.0, t_tol=1e9)
    ref = M.integrate(phi, wl.dt)
    assert not mapped.any()
    assert np.array_equal(out, ref[0]) and np.array_equal(na, ref[2]) and np.array_equal(st, ref[4])


def test_zonal_reference_is_the_first_zone_cell_and_t_tol_is_inclusive(tmp_path):
    wl, M, c, yf, yo, phi = _zonal_case(tmp_path)
    air = phi[0].copy()
    air[2:] = 1e-12
    air[2:] += yo
    air[2:] /= air[2:].sum()
    air[0] = 1500.0
    for i, dT in ((3, 0.0), (5, 2.0), (7, -2.0), (9, 2.5)):
        phi[i] = air
        phi[i, 0] += dT
    out, h, na, nr, st, mapped = M.integrate_zonal(phi, wl.dt, c, yf, yo, z_max=1e-6, t_tol=2.0)
    z = M.mixture_fraction(c, yf, yo, phi)
    assert set(np.nonzero(z <= 1e-6)[0]) == {3, 5, 7, 9}
    assert list(np.nonzero(mapped)[0]) == [5, 7]          # 3 is the reference, 9 is 2.5 K away
    solved = M.integrate(phi[mapped == 0], wl.dt)
    assert np.array_equal(out[mapped == 0], solved[0])
    for i in (5, 7):
        assert np.array_equal(out[i, 2:], phi[i, 2:] + (out[3, 2:] - phi[3, 2:]))
        assert out[i, 0] == phi[i, 0] + (out[3, 0] - phi[3, 0]) and out[i, 1] == phi[i, 1]
        assert na[i] == 0 and nr[i] == 0 and st[i] == st[3]
    # a mapped cell identical to its reference ends where integrating it would
    phi[5, 0] = phi[3, 0]
    out2, _, _, _, _, mapped2 = M.integrate_zonal(phi, wl.dt, c, yf, yo, z_max=1e-6, t_tol=2.0)
    assert mapped2[5]
    direct = M.integrate(phi[5:6], wl.dt)[0][0]
    assert np.allclose(out2[5], direct, rtol=1e-14, atol=1e-20)


def test_zonal_bands_each_have_their_own_reference(tmp_path):
    """Two Z bands (dz = 0.05): air cells (Z ~ 0) and cells of a fuel blend at
    Z ~ 0.12, each band mapped from its own first cell, with every other cell
    fuel-rich (Z ~ 0.5, outside the zone); a band width above z_max is the
    single band of dz = 0."""
    wl, M, c, yf, yo, phi = _zonal_case(tmp_path)
    air = np.full(phi.shape[1] - 2, 1e-12) + yo
    air /= air.sum()
    blend = 0.12 * yf + 0.88 * yo + 1e-12
    blend /= blend.sum()
    rich = 0.5 * yf + 0.5 * yo + 1e-12
    rich /= rich.sum()
    comp = {i: rich for i in range(phi.shape[0])}
    comp.update({2: air, 4: blend, 6: air, 8: blend, 10: blend})
    for i, y in comp.items():
        phi[i, 2:] = y
        phi[i, 0] = 1200.0 + 0.1 * i
    z = M.mixture_fraction(c, yf, yo, phi)
    assert z[2] < 1e-6 and 0.1 < z[4] < 0.15 and (z[[0, 1, 3, 5, 7, 9, 11]] > 0.4).all()
    out, h, na, nr, st, mapped = M.integrate_zonal(phi, wl.dt, c, yf, yo, z_max=0.2, t_tol=2.0, dz=0.05)
    band4 = int(np.floor(z[4] / 0.05)) + 1
    assert list(mapped) == [0, 0, 0, 0, 0, 0, 1, 0, band4, 0, band4, 0]
    for i, ref in ((6, 2), (8, 4), (10, 4)):
        assert np.array_equal(out[i, 2:], phi[i, 2:] + (out[ref, 2:] - phi[ref, 2:]))
        assert out[i, 0] == phi[i, 0] + (out[ref, 0] - phi[ref, 0])
    # one band over the same zone: every zone cell maps from cell 2
    one = M.integrate_zonal(phi, wl.dt, c, yf, yo, z_max=0.2, t_tol=2.0, dz=0.0)
    assert list(np.nonzero(one[5])[0]) == [4, 6, 8, 10]
    wide = M.integrate_zonal(phi, wl.dt, c, yf, yo, z_max=0.2, t_tol=2.0, dz=1.0)
    assert np.array_equal(wide[5], one[5]) and np.array_equal(wide[0], one[0])
