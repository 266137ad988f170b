"""The GPU right-hand side against closed forms of the rate laws, through the
C ABI (not only against the oracle): modified-Arrhenius temperature
dependence, non-unit third-body efficiencies and Troe broadening away from
Fcent = 1, on the hand-built mechanisms that pin the oracle.

For a single irreversible reaction with reactants 0 and 1 the production
rate of species 0 is -q, so f_Y0 = -W_0 q / rho with q in closed form.
"""
import math

import numpy as np
import pytest
import torch

from paper_2112_05834_amd import chem, synth
from tests import mechs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
R_GAS = 8.314462618


def _f(mech, path, states):
    phi = np.array([[T, p] + list(Y) for T, p, Y in states], dtype=np.float64)
    S = chem.Solver(chem.Mechanism(path), device=0)
    f, _ = S.eval_rhs_jac(torch.from_numpy(phi).to(DEV), jac=False)
    torch.cuda.synchronize()
    return f.cpu().numpy()


def _rho_c(mech, T, p, Y):
    Y = np.asarray(Y)
    Wbar = 1.0 / np.sum(Y / mech.W)
    rho = p * Wbar / (R_GAS * T)
    return rho, rho * Y / mech.W


def test_gpu_third_body_nonunit_efficiencies(tmp_path):
    mech = mechs.third_body_efficiencies(A=1.0e2)
    path = synth.write_mech(mech, str(tmp_path / "tbeff.mech"))
    states = [(1500.0, 3.0e5, [0.2, 0.3, 0.1, 0.4]), (900.0, 6.0e6, [0.05, 0.15, 0.5, 0.3]),
              (2400.0, 1.0e4, [0.4, 0.1, 0.3, 0.2])]
    f = _f(mech, path, states)
    for c, (T, p, Y) in enumerate(states):
        rho, C = _rho_c(mech, T, p, Y)
        q = 1.0e2 * (p / (R_GAS * T) - C[2] + 2.0 * C[3]) * C[0] * C[1]
        expect = -mech.W[0] * q / rho
        assert abs(f[c, 1] - expect) <= 1e-13 * abs(expect), (c, f[c, 1] / expect - 1)


@pytest.mark.parametrize("T", [650.0, 1100.0, 1800.0, 2600.0])
def test_gpu_troe_broadening_closed_form_points(T, tmp_path):
    """F = Fcent at X = 0 and F = Fcent^(1/2) at X = N/(1+d), with a, T3, T1,
    T2, b, Ea, b0, Ea0 and two non-unit efficiencies all active."""
    kw = dict(A=3.0e6, b=0.7, Ea=2.2e4, A0=5.0e3, b0=-1.3, Ea0=9.0e3, a=0.62, T3=170.0, T1=1900.0,
              T2=4300.0)
    mech = mechs.troe_general(**kw)
    path = synth.write_mech(mech, str(tmp_path / "troe.mech"))
    Y = np.array([0.3, 0.25, 0.15, 0.3])
    Fc = (1 - kw["a"]) * math.exp(-T / kw["T3"]) + kw["a"] * math.exp(-T / kw["T1"]) + math.exp(-kw["T2"] / T)
    L = math.log10(Fc)
    c, N, d = -0.4 - 0.67 * L, 0.75 - 1.27 * L, 0.14
    kinf = kw["A"] * T ** kw["b"] * math.exp(-kw["Ea"] / (R_GAS * T))
    k0 = kw["A0"] * T ** kw["b0"] * math.exp(-kw["Ea0"] / (R_GAS * T))
    X = (Y / mech.W) / np.sum(Y / mech.W)
    m_per_ctot = 1.0 - X[2] + 2.0 * X[3]
    states, expect = [], []
    for logPr, F in [(0.4 + 0.67 * L, Fc), (N / (1.0 + d) - c, math.sqrt(Fc))]:
        Pr = 10.0 ** logPr
        p = Pr * kinf / k0 / m_per_ctot * R_GAS * T
        rho, C = _rho_c(mech, T, p, Y)
        states.append((T, p, Y))
        expect.append(-mech.W[0] * kinf * Pr / (1.0 + Pr) * F * C[0] * C[1] / rho)
    f = _f(mech, path, states)
    for c_, e in enumerate(expect):
        assert abs(f[c_, 1] - e) <= 1e-12 * abs(e), (T, c_, f[c_, 1] / e - 1)


def test_gpu_arrhenius_temperature_dependence(tmp_path):
    """A <=> B isomers with kf = A T^b exp(-Ea/(RT)) (b, Ea != 0) and
    kr = kf exp(-shift): f_YA = -(kf Y_A - kr Y_B) at every T (equal W, so
    W/rho C = Y). The ratio of f at three temperatures recovers b and Ea/R."""
    A, b, Ea, shift = 4.0e9, 1.7, 8.5e4, 0.45
    mech = mechs.arrhenius_isomer(A, b, Ea, shift)
    path = synth.write_mech(mech, str(tmp_path / "arr.mech"))
    Ts = [300.0, 700.0, 1000.0, 1300.0, 2400.0, 5000.0]
    Y = [0.7, 0.3]
    f = _f(mech, path, [(T, 1e5, Y) for T in Ts])
    lk = []
    for c, T in enumerate(Ts):
        kf = A * T ** b * math.exp(-Ea / (R_GAS * T))
        kr = kf * math.exp(-shift)
        expect = -(kf * Y[0] - kr * Y[1])
        assert abs(f[c, 1] - expect) <= 1e-13 * abs(expect), (T, f[c, 1] / expect - 1)
        assert f[c, 0] == 0.0 or abs(f[c, 0]) <= 1e-9 * abs(expect)     # dH = 0: T does not move
        lk.append(math.log(-f[c, 1] / (Y[0] - math.exp(-shift) * Y[1])))
    G = np.stack([np.ones(3), np.log(Ts[1::2]), -1.0 / np.array(Ts[1::2])], axis=1)
    x = np.linalg.solve(G, np.array(lk[1::2]))
    ex = np.array([math.log(A), b, Ea / R_GAS])
    assert np.all(np.abs(x - ex) <= 1e-11 * np.abs(ex)), x - ex
