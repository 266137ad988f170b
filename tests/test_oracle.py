"""Pins of the CPU oracle against mathematics (not against itself).

Each test names what fixes the expected value: an exact property of the
Rodas3 tableau, a closed-form solution of a hand-built mechanism, a
finite-difference derivative, LAPACK (via scipy), an independent stiff solver
(scipy Radau), or a conservation law of the model equations.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

from oracle import oracle as O
from paper_2112_05834_amd import synth
from tests import mechs

R_GAS = 8.314462618
P_ATM = 101325.0


def _write(m, d, name):
    return synth.write_mech(m, "%s/%s.mech" % (d, name))


# ---------------------------------------------------------------- Rodas3 ---

def _tableau_fractions():
    g, a, c, m, e = O.rodas3_tableau()
    F = lambda x: Fraction(x).limit_denominator(1000)
    gam = F(g)
    A = [[F(a[i, j]) for j in range(4)] for i in range(4)]
    C = [[F(c[i, j]) for j in range(4)] for i in range(4)]
    M = [F(x) for x in m]
    E = [F(x) for x in e]
    # the doubles must be exactly these rationals (up to the rounding of -8/3)
    for x, fx in [(g, gam)] + [(a[i, j], A[i][j]) for i in range(4) for j in range(4)] \
            + [(c[i, j], C[i][j]) for i in range(4) for j in range(4)]:
        assert float(fx) == x
    return gam, A, C, M, E


def _linear_stages(gam, A, C, M, E, z):
    """Rodas3 on y' = lambda y, y0 = 1, at z = h lambda, in exact arithmetic:
    (1/gamma - z) K_i = z (1 + sum a_ij K_j) + sum c_ij K_j."""
    K = []
    for i in range(4):
        r = z * (1 + sum(A[i][j] * K[j] for j in range(i))) + sum(C[i][j] * K[j] for j in range(i))
        K.append(r / (1 / gam - z))
    R = 1 + sum(M[j] * K[j] for j in range(4))
    Err = sum(E[j] * K[j] for j in range(4))
    return R, Err


def _R_closed(z):
    # stability function of Rodas3 (order 3, L-stable)
    return Fraction(8) * (z ** 3 - 6 * z + 6) / (3 * (z - 2) ** 4)


def _Rhat_closed(z):
    # stability function of the embedded order-2 solution
    return Fraction(2) * (z ** 2 + 2 * z - 4) / (z - 2) ** 3


def test_rodas3_stability_function_closed_form():
    tab = _tableau_fractions()
    for z in [Fraction(-1, 3), Fraction(1, 7), Fraction(-5), Fraction(-1000), Fraction(3, 2)]:
        R, Err = _linear_stages(*tab, z)
        assert R == _R_closed(z)
        assert R - Err == _Rhat_closed(z)


def test_rodas3_order_on_linear_problem():
    """R(z) - e^z = O(z^4) and Rhat(z) - e^z = O(z^3), exactly: compare
    Taylor coefficients of the exact rational functions."""
    tab = _tableau_fractions()
    # Taylor coefficients by exact evaluation at tiny z with Richardson-free
    # algebra: R(z) is rational; expand via sympy-free finite differences of
    # exact values is awkward, so check the defect ratio instead.
    for order, f in [(3, lambda z: _linear_stages(*tab, z)[0]),
                     (2, lambda z: (lambda R, E: R - E)(*_linear_stages(*tab, z)))]:
        defects = []
        for k in range(4, 9):
            z = Fraction(1, 2 ** k)
            ez = sum(z ** j / math.factorial(j) for j in range(12))
            defects.append(abs(f(z) - ez))
        ratios = [float(defects[i] / defects[i + 1]) for i in range(len(defects) - 1)]
        # defect ~ z^(order+1): halving z divides it by 2^(order+1)
        for r in ratios[1:]:
            assert abs(r - 2 ** (order + 1)) / 2 ** (order + 1) < 0.1


def test_rodas3_L_stable():
    tab = _tableau_fractions()
    R, _ = _linear_stages(*tab, Fraction(-10) ** 12)
    assert abs(float(R)) < 1e-11


def test_rodas3_nonlinear_order_conditions():
    """Order-3 conditions of the classical form, derived from the transformed
    coefficients: Gamma from gamma and c, alpha from a."""
    gam, A, C, M, E = _tableau_fractions()
    # transformed form: a = alpha Gamma^-1, c = diag(1/gamma) - Gamma^-1, m = b Gamma^-1
    # so Gamma^-1 = diag(1/gamma) - c, alpha = a Gamma, b = m Gamma.
    Ginv = [[(1 / gam if i == j else 0) - C[i][j] for j in range(4)] for i in range(4)]
    G = _inv_lower(Ginv)
    alpha = [[sum(A[i][k] * G[k][j] for k in range(4)) for j in range(4)] for i in range(4)]
    b = [sum(M[k] * G[k][j] for k in range(4)) for j in range(4)]
    al = [sum(alpha[i][j] for j in range(4)) for i in range(4)]
    # beta_ij = alpha_ij + gamma_ij; beta'_i = sum_{j<i} beta_ij
    beta_p = [sum(alpha[i][j] + G[i][j] for j in range(i)) for i in range(4)]
    assert sum(b) == 1
    assert sum(b[i] * beta_p[i] for i in range(4)) == Fraction(1, 2) - gam
    assert sum(b[i] * al[i] ** 2 for i in range(4)) == Fraction(1, 3)
    bb = sum(b[i] * sum((alpha[i][k] + G[i][k]) * beta_p[k] for k in range(i)) for i in range(4))
    assert bb == Fraction(1, 6) - gam + gam ** 2
    # stiff accuracy: b equals the last row of alpha + Gamma
    assert b == [alpha[3][j] + G[3][j] for j in range(4)]


def _inv_lower(L):
    n = len(L)
    X = [[Fraction(0)] * n for _ in range(n)]
    for j in range(n):
        for i in range(n):
            s = Fraction(1 if i == j else 0) - sum(L[i][k] * X[k][j] for k in range(i))
            X[i][j] = s / L[i][i]
    return X


# ------------------------------------------------- closed-form mechanisms ---

def test_one_step_isomer_matches_stability_function(mech_dir):
    kf = 2.0e5
    shift = 0.7
    M = O.Mech(_write(mechs.isomer_pair(kf, shift), mech_dir, "iso"))
    kr = kf / math.exp(shift)
    yeq = kr / (kf + kr)
    tab = _tableau_fractions()
    for h in [1e-7, 3e-6, 1e-4, 1e-2]:
        y0 = np.array([1200.0, 0.9, 0.1])
        yn, err = M.rodas3_step(1e5, y0, h)
        z = Fraction(-(kf + kr) * h)
        R, E = _linear_stages(*tab, z)
        d0 = y0[1] - yeq
        assert yn[0] == y0[0]
        assert abs((yn[1] - yeq) - float(R) * d0) <= 1e-13 * abs(d0)
        assert abs(err[1] - float(E) * d0) <= 1e-13 * abs(d0)
        assert abs(yn[1] + yn[2] - 1.0) < 1e-13


def test_adaptive_isomer_closed_form(mech_dir):
    kf, shift = 2.0e5, 0.7
    M = O.Mech(_write(mechs.isomer_pair(kf, shift), mech_dir, "iso2"))
    kr = kf / math.exp(shift)
    yeq = kr / (kf + kr)
    phi = np.array([[1100.0, 1e5, 0.95, 0.05], [900.0, 1e5, 0.0, 1.0]])
    for dt in [1e-6, 1e-5, 1e-4]:
        out, h, na, nr, st = M.integrate(phi, dt)
        assert (st == 0).all()
        ya = yeq + (phi[:, 2] - yeq) * math.exp(-(kf + kr) * dt)
        assert np.all(np.abs(out[:, 2] - ya) <= 10 * (1e-10 + 1e-6 * np.abs(ya)))
        assert np.all(out[:, 0] == phi[:, 0])


def test_convergence_order_termolecular(mech_dir):
    """Fixed-step Rodas3 on 3A -> 3B: global error of the main solution falls
    as h^3, of the embedded solution as h^2."""
    k = 1.0e2
    mech = mechs.termolecular_isomer(k)
    M = O.Mech(_write(mech, mech_dir, "ter"))
    T, p = 1000.0, 1.0e5
    y0 = np.array([T, 1.0, 0.0])
    C0 = p / (R_GAS * T)
    rho = p * mech.W[0] / (R_GAS * T)
    t_end = 2.0 / (k * C0 * C0)
    exact = C0 / math.sqrt(1 + 6 * k * C0 * C0 * t_end) * mech.W[0] / rho
    errs_main, errs_emb = [], []
    for N in [32, 64, 128, 256, 512, 1024]:
        h = t_end / N
        y, ye = y0.copy(), y0.copy()
        for _ in range(N):
            y, _ = M.rodas3_step(p, y, h)
            yn, e = M.rodas3_step(p, ye, h)
            ye = yn - e
        errs_main.append(abs(y[1] - exact))
        errs_emb.append(abs(ye[1] - exact))
    sm = [math.log2(errs_main[i] / errs_main[i + 1]) for i in range(4)]
    se = [math.log2(errs_emb[i] / errs_emb[i + 1]) for i in range(5)]
    assert abs(sm[-1] - 3.0) < 0.1 and abs(sm[-2] - 3.0) < 0.1, sm
    assert abs(se[-1] - 2.0) < 0.05 and abs(se[-2] - 2.0) < 0.1, se


def test_third_body_unit_efficiencies(mech_dir):
    mech = mechs.third_body_unit(A=1.0e2)
    M = O.Mech(_write(mech, mech_dir, "tb"))
    T, p = 1500.0, 3.0e5
    Y = np.array([0.2, 0.3, 0.1, 0.4])
    kf, kr, q = M.rates(T, p, Y)
    Wbar = 1.0 / np.sum(Y / mech.W)
    rho = p * Wbar / (R_GAS * T)
    C = rho * Y / mech.W
    expect = 1.0e2 * (p / (R_GAS * T)) * C[0] * C[1]
    assert kr[0] == 0.0
    assert abs(q[0] - expect) <= 4e-15 * abs(expect)


def test_troe_reduces_to_lindemann(mech_dir):
    A, A0 = 1.0e7, 1.0e4
    mech = mechs.troe_lindemann(A, A0)
    M = O.Mech(_write(mech, mech_dir, "lind"))
    for T, p in [(1200.0, 1e5), (2000.0, 6e6), (800.0, 1e3)]:
        Y = np.array([0.25, 0.25, 0.2, 0.3])
        kf, kr, q = M.rates(T, p, Y)
        Wbar = 1.0 / np.sum(Y / mech.W)
        rho = p * Wbar / (R_GAS * T)
        C = rho * Y / mech.W
        Mconc = p / (R_GAS * T)
        Pr = A0 * Mconc / A
        expect = A * Pr / (1 + Pr) * C[0] * C[1]
        assert abs(q[0] - expect) <= 1e-14 * abs(expect)


def _conc(mech, T, p, Y):
    Wbar = 1.0 / np.sum(Y / mech.W)
    rho = p * Wbar / (R_GAS * T)
    return rho * Y / mech.W


def test_third_body_nonunit_efficiencies(mech_dir):
    """Efficiency 0 for species 2 and 3 for species 3 (all others 1): the
    third-body concentration is p/(RT) - C_2 + 2 C_3, so a wrong species index
    in the efficiency lookup, or an efficiency applied as alpha - 1 twice,
    moves q off the closed form."""
    mech = mechs.third_body_efficiencies(A=1.0e2)
    M = O.Mech(_write(mech, mech_dir, "tbeff"))
    for T, p, Y in [(1500.0, 3.0e5, [0.2, 0.3, 0.1, 0.4]), (900.0, 6.0e6, [0.05, 0.15, 0.5, 0.3]),
                    (2400.0, 1.0e4, [0.4, 0.1, 0.3, 0.2])]:
        Y = np.array(Y)
        C = _conc(mech, T, p, Y)
        Mconc = p / (R_GAS * T) - C[2] + 2.0 * C[3]
        _, kr, q = M.rates(T, p, Y)
        expect = 1.0e2 * Mconc * C[0] * C[1]
        assert kr[0] == 0.0
        assert abs(q[0] - expect) <= 1e-14 * abs(expect), (T, p)


def _troe_fcent(a, T3, T1, T2, T):
    return (1.0 - a) * math.exp(-T / T3) + a * math.exp(-T / T1) + math.exp(-T2 / T)


@pytest.mark.parametrize("T", [650.0, 1100.0, 1800.0, 2600.0])
def test_troe_broadening_closed_form_points(T, mech_dir):
    """Troe falloff with a, T3, T1 and T2 all active (Fcent away from 1),
    both rate constants with b != 0 and Ea != 0, and efficiencies 0 and 3.

    With L = log10 Fcent, c = -0.4 - 0.67 L, N = 0.75 - 1.27 L, d = 0.14 and
    X = log10 Pr + c, the broadening is log10 F = L / (1 + (X/(N - dX))^2).
    Two pressures are chosen for each T so that it takes closed values:
    X = 0 gives F = Fcent exactly (pins c and the T2 term), and
    X = N/(1+d) gives X/(N - dX) = 1, so F = Fcent^(1/2) (pins N and d).
    The rate of progress is then q = k_inf Pr/(1+Pr) F C_A C_B."""
    kw = dict(A=3.0e6, b=0.7, Ea=2.2e4, A0=5.0e3, b0=-1.3, Ea0=9.0e3, a=0.62, T3=170.0, T1=1900.0,
              T2=4300.0)
    mech = mechs.troe_general(**kw)
    M = O.Mech(_write(mech, mech_dir, "troegen_%d" % int(T)))
    Y = np.array([0.3, 0.25, 0.15, 0.3])
    Fc = _troe_fcent(kw["a"], kw["T3"], kw["T1"], kw["T2"], T)
    assert abs(Fc - 1.0) > 0.05          # away from the Lindemann limit
    L = math.log10(Fc)
    c, N, d = -0.4 - 0.67 * L, 0.75 - 1.27 * L, 0.14
    kinf = kw["A"] * T ** kw["b"] * math.exp(-kw["Ea"] / (R_GAS * T))
    k0 = kw["A0"] * T ** kw["b0"] * math.exp(-kw["Ea0"] / (R_GAS * T))
    # [M] = (p/(RT)) (1 - X_2 + 2 X_3) with mole fractions X, so Pr is linear in p
    X_mole = (Y / mech.W) / np.sum(Y / mech.W)
    m_per_ctot = 1.0 - X_mole[2] + 2.0 * X_mole[3]
    for logPr, F_exp in [(0.4 + 0.67 * L, Fc), (N / (1.0 + d) - c, math.sqrt(Fc))]:
        Pr = 10.0 ** logPr
        p = Pr * kinf / k0 / m_per_ctot * R_GAS * T
        C = _conc(mech, T, p, Y)
        expect = kinf * Pr / (1.0 + Pr) * F_exp * C[0] * C[1]
        kf, kr, q = M.rates(T, p, Y)
        assert abs(kf[0] - kinf) <= 1e-14 * kinf
        assert kr[0] == 0.0
        assert abs(q[0] - expect) <= 1e-12 * abs(expect), (T, logPr, q[0] / expect - 1.0)


def test_arrhenius_temperature_dependence_recovered(mech_dir):
    """kf = A T^b exp(-Ea/(RT)) with b != 0 and Ea != 0: ln kf at three
    temperatures determines (ln A, b, Ea/R) through an exact 3x3 solve of
    ln kf = ln A + b ln T - (Ea/R)/T. A units slip in Ea or R, or a wrong sign
    of b, moves the recovered triple off the file's values. For the isomer
    pair Kc = exp(a7_B - a7_A) does not depend on T, so ln kr recovers the
    same b and Ea/R with ln A lowered by the a7 shift."""
    A, b, Ea, shift = 4.0e9, 1.7, 8.5e4, 0.45
    mech = mechs.arrhenius_isomer(A, b, Ea, shift)
    M = O.Mech(_write(mech, mech_dir, "arr"))
    expect = np.array([math.log(A), b, Ea / R_GAS])
    for Ts in ([700.0, 1300.0, 2400.0], [300.0, 1000.0, 5000.0]):
        Ts = np.array(Ts)
        lkf, lkr = [], []
        for T in Ts:
            kf, kr, _ = M.rates(T, 1e5, np.array([0.5, 0.5]))
            lkf.append(math.log(kf[0]))
            lkr.append(math.log(kr[0]))
        G = np.stack([np.ones(3), np.log(Ts), -1.0 / Ts], axis=1)
        xf = np.linalg.solve(G, np.array(lkf))
        xr = np.linalg.solve(G, np.array(lkr))
        assert np.all(np.abs(xf - expect) <= 1e-12 * np.abs(expect)), xf - expect
        assert np.all(np.abs(xr - (expect - [shift, 0.0, 0.0])) <= 1e-12 * np.abs(expect)), xr - expect


def test_thermo_derivatives(mech_dir):
    mech, path = synth.mech_cached("spray54", mech_dir)
    M = O.Mech(path)
    for T in [350.0, 900.0, 1700.0, 3100.0]:
        cp, h, s, dcp = M.thermo(T)
        d = 1e-3
        _, hp, sp, _ = M.thermo(T + d)
        _, hm, sm, _ = M.thermo(T - d)
        cpp, _, _, _ = M.thermo(T + d)
        cpm, _, _, _ = M.thermo(T - d)
        dH = (hp * (T + d) - hm * (T - d)) / (2 * d)     # d(h/R)/dT = cp/R
        dS = (sp - sm) / (2 * d)                          # d(s/R)/dT = cp/(R T)
        assert np.allclose(dH, cp, rtol=1e-9, atol=0)
        assert np.allclose(dS, cp / T, rtol=1e-8, atol=0)
        assert np.allclose((cpp - cpm) / (2 * d), dcp, rtol=1e-6, atol=1e-12)


def test_equilibrium_constant_isomer(mech_dir):
    shift = 0.37
    M = O.Mech(_write(mechs.isomer_pair(1e3, shift), mech_dir, "iso3"))
    kf, kr, _ = M.rates(1500.0, 1e5, np.array([0.5, 0.5]))
    assert abs(kf[0] / kr[0] - math.exp(shift)) < 1e-14 * math.exp(shift)


def test_irreversible_has_no_reverse_rate(mech_dir):
    M = O.Mech(_write(mechs.isomer_pair(1e3, 0.3, reversible=False), mech_dir, "iso4"))
    kf, kr, q = M.rates(1500.0, 1e5, np.array([0.5, 0.5]))
    assert kr[0] == 0.0 and kf[0] == 1e3


# --------------------------------------------------------------- Jacobian ---

def fd_jacobian_check(M, p, y, floorT=1.0, floorY=1e-8):
    """Central-difference check in the scaled form diag(1/s) J diag(s)."""
    n = len(y)
    s = np.abs(y).copy()
    s[0] = max(s[0], floorT)
    s[1:] = np.maximum(s[1:], floorY)
    J = M.jac(p, y)
    Jfd = np.zeros_like(J)
    for j in range(n):
        d = 1e-6 * s[j]
        yp, ym = y.copy(), y.copy()
        yp[j] += d
        ym[j] -= d
        Jfd[:, j] = (M.rhs(p, yp) - M.rhs(p, ym)) / (2 * d)
    Ja = J * s[None, :] / s[:, None]
    Jf = Jfd * s[None, :] / s[:, None]
    rowmax = np.abs(Ja).max(axis=1, keepdims=True)
    bad = np.abs(Ja - Jf) > 1e-6 * np.abs(Jf) + 1e-9 * rowmax
    return int(bad.sum())


@pytest.mark.parametrize("name", ["tiny9_1024", "spray54_262144"])
def test_jacobian_vs_finite_differences(name, mech_dir):
    wl, mech, path, phi = synth.workload_inputs(name, mech_dir, n_cells=2000)
    M = O.Mech(path)
    idx = synth.sample_indices(phi.shape[0], 12, 11)
    for c in idx:
        y = np.concatenate([[phi[c, 0]], phi[c, 2:]])
        assert fd_jacobian_check(M, phi[c, 1], y) == 0


def test_jacobian_falloff_chain_rule(mech_dir):
    mech = mechs.troe_mix()
    M = O.Mech(_write(mech, mech_dir, "troemix"))
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(20):
        T = rng.uniform(600, 2800)
        p = 10 ** rng.uniform(3.5, 7)
        Y = rng.dirichlet(np.ones(mech.n_species))
        y = np.concatenate([[T], Y])
        assert fd_jacobian_check(M, p, y, floorY=1e-6) == 0


# --------------------------------------------------------------------- LU ---

def test_lu_matches_lapack():
    rng = np.random.Generator(np.random.PCG64(1))
    for n in [1, 2, 10, 55, 161]:
        A = rng.normal(size=(n, n)) + n ** 0.5 * np.eye(n) * rng.uniform(0, 1)
        LU, piv, info = O.lu(A)
        lu_ref, piv_ref = scipy.linalg.lu_factor(A)
        assert info == 0
        assert np.array_equal(piv, piv_ref)
        assert np.max(np.abs(LU - lu_ref)) <= 1e-12 * np.max(np.abs(A))
        b = rng.normal(size=n)
        x = O.lu_solve(LU, piv, b)
        x_ref = scipy.linalg.lu_solve((lu_ref, piv_ref), b)
        assert np.max(np.abs(x - x_ref)) <= 1e-11 * np.max(np.abs(x_ref))


def test_lu_on_integrator_matrix(mech_dir):
    wl, mech, path, phi = synth.workload_inputs("spray54_262144", mech_dir, n_cells=64)
    M = O.Mech(path)
    for c in range(0, 64, 9):
        y = np.concatenate([[phi[c, 0]], phi[c, 2:]])
        J = M.jac(phi[c, 1], y)
        A = np.eye(M.n) / (0.5 * 1e-8) - J
        LU, piv, info = O.lu(A)
        lu_ref, piv_ref = scipy.linalg.lu_factor(A)
        assert np.array_equal(piv, piv_ref)
        b = np.arange(M.n, dtype=float) + 1
        x = O.lu_solve(LU, piv, b)
        r = A @ x - b
        assert np.max(np.abs(r)) <= M.n * 1e-15 * np.max(np.abs(A)) * np.max(np.abs(x)) * 10


def test_lu_singular_reports_column():
    A = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [1.0, 0.0, 1.0]])
    _, _, info = O.lu(A)
    assert info == 3


# ------------------------------------------------------------- integrator ---

def _element_totals(mech, Y):
    return (Y / mech.W) @ mech.elem


def _enthalpy(M, mech, T, Y):
    out = np.empty(len(T))
    for c in range(len(T)):
        _, h, _, _ = M.thermo(T[c])
        out[c] = np.sum(Y[c] * h * R_GAS * T[c] / mech.W)
    return out


def test_invariants_tiny9(mech_dir):
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", mech_dir)
    M = O.Mech(path)
    out, h, na, nr, st = M.integrate(phi, wl.dt, n_threads=8)
    assert (st == 0).all()
    e0 = _element_totals(mech, phi[:, 2:])
    e1 = _element_totals(mech, out[:, 2:])
    used = e0.max(axis=0) > 0
    rel = np.abs(e1 - e0)[:, used] / e0[:, used].max(axis=1, keepdims=True)
    assert rel.max() <= 1e-12
    assert np.abs(out[:, 2:].sum(axis=1) - 1.0).max() <= 1e-13
    assert np.all(out[:, 1] == phi[:, 1])
    H0 = _enthalpy(M, mech, phi[:, 0], phi[:, 2:])
    H1 = _enthalpy(M, mech, out[:, 0], out[:, 2:])
    cpT = np.array([np.sum(phi[c, 2:] * M.thermo(phi[c, 0])[0] * R_GAS / mech.W) * phi[c, 0] for c in range(64)])
    assert np.all(np.abs(H1[:64] - H0[:64]) <= 10 * 1e-6 * cpT)


def test_entropy_non_decreasing(mech_dir):
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", mech_dir, n_cells=16)
    M = O.Mech(path)

    def s_mix(T, p, Y):
        _, _, s, _ = M.thermo(T)
        X = (Y / mech.W) / np.sum(Y / mech.W)
        return np.sum(Y / mech.W * R_GAS * (s - np.log(X * p / P_ATM)))

    cur = phi.copy()
    h = None
    for _ in range(8):
        nxt, h, na, nr, st = M.integrate(cur, 2e-7, h_io=h)
        for c in range(cur.shape[0]):
            if (cur[c, 2:] > 0).all() and (nxt[c, 2:] > 0).all():
                s0 = s_mix(cur[c, 0], cur[c, 1], cur[c, 2:])
                s1 = s_mix(nxt[c, 0], nxt[c, 1], nxt[c, 2:])
                assert s1 - s0 >= -1e-9 * abs(s0)
        cur = nxt


def test_equilibrium_isomer_cycle(mech_dir):
    """Detailed balance: at X_i ~ exp(a7_i) every reaction has Q_r = Kc_r, so
    f = 0 and integration leaves the state alone; from elsewhere the
    integrator converges to that state."""
    shifts = (0.0, 0.9, -0.4)
    M = O.Mech(_write(mechs.isomer_cycle(shifts), mech_dir, "cyc"))
    yeq = np.exp(shifts) / np.sum(np.exp(shifts))
    y = np.concatenate([[1500.0], yeq])
    f = M.rhs(1e5, y)
    kf, kr, q = M.rates(1500.0, 1e5, yeq)
    C = 1e5 / (R_GAS * 1500.0) * yeq
    assert np.all(np.abs(q) <= 1e-13 * kf * C.max())
    assert np.all(np.abs(f[1:]) <= 1e-13 * kf.max())
    phi = np.array([[1500.0, 1e5, *yeq], [1500.0, 1e5, 1.0, 0.0, 0.0], [1500.0, 1e5, 0.1, 0.2, 0.7]])
    out, h, na, nr, st = M.integrate(phi, 1e-3, rtol=1e-10, atol=1e-16)
    assert (st == 0).all()
    assert np.max(np.abs(out[0, 2:] - yeq)) <= 1e-14
    assert np.max(np.abs(out[1:, 2:] - yeq)) <= 1e-9


def test_equilibrium_dissociation(mech_dir):
    mech = mechs.dissociation()
    M = O.Mech(_write(mech, mech_dir, "diss"))
    T, p = 2500.0, 2e5
    cp, h, s, _ = M.thermo(T)
    assert abs(h[0] - 2 * h[1]) <= 1e-14 * abs(h[0])
    g = h - s
    Kc = math.exp(-(2 * g[1] - g[0])) * (P_ATM / (R_GAS * T))
    Ctot = p / (R_GAS * T)
    CB = (-Kc + math.sqrt(Kc * Kc + 4 * Kc * Ctot)) / 2
    CA = Ctot - CB
    YA = CA * mech.W[0] / (CA * mech.W[0] + CB * mech.W[1])
    phi = np.array([[T, p, 1.0, 0.0], [T, p, 0.3, 0.7]])
    out, hh, na, nr, st = M.integrate(phi, 1e-3, rtol=1e-10, atol=1e-16)
    assert (st == 0).all()
    assert np.all(np.abs(out[:, 0] - T) <= 1e-9 * T)
    assert np.max(np.abs(out[:, 2] - YA)) <= 1e-8


def test_thermo_matches_construction(mech_dir):
    """NASA values reproduce the generator's defining draws: cp/R is the
    smoothstep closed form, h/R(T) - a6 is the integral of cp/R from 0, and
    s/R(298.15) is the drawn standard entropy."""
    import scipy.integrate as si
    cp0, dcp, a6, s298 = 4.2, 1.3, -1234.5, 31.0
    nasa = synth.nasa_from_draws(cp0, dcp, a6, s298)
    mech = mechs._mech([(1, 1, 0, 0)], [nasa], [], names=["X"])
    M = O.Mech(_write(mech, mech_dir, "one"))
    cp_true = lambda T: cp0 + dcp * (3 * ((T - 200) / 5800) ** 2 - 2 * ((T - 200) / 5800) ** 3)
    for T in [250.0, 700.0, 1000.0, 2345.0, 5900.0]:
        cp, h, s, _ = M.thermo(T)
        assert abs(cp[0] - cp_true(T)) <= 1e-12 * cp_true(T)
        integral, _ = si.quad(cp_true, 0.0, T, epsabs=0, epsrel=1e-13)
        assert abs(h[0] * T - a6 - integral) <= 1e-9 * abs(integral)
    _, _, s, _ = M.thermo(298.15)
    assert abs(s[0] - s298) <= 1e-12 * s298


def test_integrator_vs_scipy_radau(mech_dir):
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", mech_dir, n_cells=512)
    M = O.Mech(path)
    idx = synth.sample_indices(512, 6, 5)
    out, h, na, nr, st = M.integrate(phi[idx], wl.dt)
    for k, c in enumerate(idx):
        p = phi[c, 1]
        y0 = np.concatenate([[phi[c, 0]], phi[c, 2:]])
        sol = scipy.integrate.solve_ivp(lambda t, y: M.rhs(p, y), (0.0, wl.dt), y0, method="Radau",
                                        jac=lambda t, y: M.jac(p, y), rtol=1e-12, atol=1e-16)
        assert sol.success
        yref = sol.y[:, -1]
        mine = np.concatenate([[out[k, 0]], out[k, 2:]])
        assert np.all(np.abs(mine - yref) <= 10 * (1e-10 + 1e-6 * np.abs(yref)))


def test_status_codes(mech_dir):
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", mech_dir, n_cells=4)
    M = O.Mech(path)
    bad = phi.copy()
    bad[0, 3] = np.nan
    bad[1, 0] = 199.0
    bad[1, 2:] = 0.0
    bad[1, 2 + mech.inert] = 1.0           # inert gas: T stays at 199 K
    out, h, na, nr, st = M.integrate(bad, wl.dt)
    assert st[0] == 3 and np.isnan(out[0, 3])
    assert st[1] == 5 and out[1, 0] == 199.0
    out, h, na, nr, st = M.integrate(phi, wl.dt, max_steps=1)
    assert (st == 1).all() or ((st == 1) | (st == 0)).all()
    assert (st[na + nr >= 1] >= 0).all()
    out, h, na, nr, st = M.integrate(phi[2:], wl.dt, rtol=1e-30, atol=1e-300)
    assert (st == 2).all()
    assert (na == 0).all()
    assert np.array_equal(out, phi[2:])


# ------------------------------------------------------- ROS4 (NEXT-4) ---
# The second scheme is a table swap: Shampine's ROS4 (order 4, embedded
# order 3, gamma = 1/2) in the same transformed form. Its pins are exact
# (rational) properties of the tableau and closed-form solutions.

def _tab_fractions(scheme):
    st, g, a, c, m, e = O.tableau(scheme)
    F = lambda x: Fraction(x).limit_denominator(1000)
    vals = [g] + list(a.ravel()) + list(c.ravel()) + list(m) + list(e)
    for x in vals:
        assert float(F(x)) == x          # every double is exactly its rational's rounding
    A = [[F(a[i, j]) for j in range(4)] for i in range(4)]
    C = [[F(c[i, j]) for j in range(4)] for i in range(4)]
    return st, F(g), A, C, [F(x) for x in m], [F(x) for x in e]


def _order_defects(gam, A, C, w):
    """Defects of the classical Rosenbrock order conditions up to order 4 for
    weights w (transformed form: Gamma^-1 = I/gamma - c, alpha = a Gamma,
    b = w Gamma). Hairer and Wanner, Solving ODEs II, Table IV.7.1."""
    s = 4
    G = _inv_lower([[(1 / gam if i == j else 0) - C[i][j] for j in range(s)] for i in range(s)])
    al = [[sum(A[i][k] * G[k][j] for k in range(s)) for j in range(s)] for i in range(s)]
    be = [[al[i][j] + G[i][j] for j in range(s)] for i in range(s)]
    b = [sum(w[k] * G[k][j] for k in range(s)) for j in range(s)]
    ai = [sum(al[i][j] for j in range(i)) for i in range(s)]
    bp = [sum(be[i][j] for j in range(i)) for i in range(s)]
    R = range(s)
    return {
        1: [sum(b) - 1],
        2: [sum(b[i] * bp[i] for i in R) - (Fraction(1, 2) - gam)],
        3: [sum(b[i] * ai[i] ** 2 for i in R) - Fraction(1, 3),
            sum(b[i] * be[i][j] * bp[j] for i in R for j in range(i)) - (Fraction(1, 6) - gam + gam ** 2)],
        4: [sum(b[i] * ai[i] ** 3 for i in R) - Fraction(1, 4),
            sum(b[i] * ai[i] * al[i][j] * bp[j] for i in R for j in range(i)) - (Fraction(1, 8) - gam / 3),
            sum(b[i] * be[i][j] * ai[j] ** 2 for i in R for j in range(i)) - (Fraction(1, 12) - gam / 3),
            sum(b[i] * be[i][j] * be[j][k] * bp[k] for i in R for j in range(i) for k in range(j))
            - (Fraction(1, 24) - gam / 2 + Fraction(3, 2) * gam ** 2 - gam ** 3)],
    }


def test_ros4_order_conditions_exact():
    st, gam, A, C, M, E = _tab_fractions(O.ROS4)
    assert st == 4 and gam == Fraction(1, 2)
    main = _order_defects(gam, A, C, M)
    emb = _order_defects(gam, A, C, [M[i] - E[i] for i in range(4)])
    for p in (1, 2, 3, 4):
        assert all(d == 0 for d in main[p]), (p, main[p])
    for p in (1, 2, 3):
        assert all(d == 0 for d in emb[p]), (p, emb[p])
    assert any(d != 0 for d in emb[4])           # the estimate is of order 3, not 4
    # the checker is not vacuous: Rodas3 meets order 3 exactly and misses 4
    _, g3, A3, C3, M3, _ = _tab_fractions(O.RODAS3)
    r3 = _order_defects(g3, A3, C3, M3)
    assert all(d == 0 for p in (1, 2, 3) for d in r3[p]) and any(d != 0 for d in r3[4])


def _ros_linear(gam, A, C, M, E, z):
    K = []
    for i in range(4):
        r = z * (1 + sum(A[i][j] * K[j] for j in range(i))) + sum(C[i][j] * K[j] for j in range(i))
        K.append(r / (1 / gam - z))
    return 1 + sum(M[j] * K[j] for j in range(4)), sum(E[j] * K[j] for j in range(4))


def test_ros4_stability_function():
    """On y' = lambda y the step multiplies y by R(z): R - e^z = O(z^5) and
    the embedded R - E - e^z = O(z^4) (halving z divides the defect by 32 and
    16); R(infinity) = 1/3, so the scheme is A-stable (|R(iy)| <= 1) but, unlike
    Rodas3, not L-stable."""
    _, gam, A, C, M, E = _tab_fractions(O.ROS4)
    for order, f in [(4, lambda z: _ros_linear(gam, A, C, M, E, z)[0]),
                     (3, lambda z: (lambda R, Er: R - Er)(*_ros_linear(gam, A, C, M, E, z)))]:
        defects = []
        for k in range(5, 10):
            z = Fraction(1, 2 ** k)
            ez = sum(z ** j / math.factorial(j) for j in range(14))
            defects.append(abs(f(z) - ez))
        ratios = [float(defects[i] / defects[i + 1]) for i in range(len(defects) - 1)]
        for r in ratios[1:]:
            assert abs(r - 2 ** (order + 1)) / 2 ** (order + 1) < 0.1, (order, ratios)
    R_inf, _ = _ros_linear(gam, A, C, M, E, Fraction(-10) ** 15)
    assert abs(float(R_inf) - 1.0 / 3.0) < 1e-12
    for k in range(1, 400):
        zz = complex(0.0, k / 4.0)
        Kc = []
        for i in range(4):
            r = zz * (1 + sum(float(A[i][j]) * Kc[j] for j in range(i))) + sum(float(C[i][j]) * Kc[j] for j in range(i))
            Kc.append(r / (float(1 / gam) - zz))
        assert abs(1 + sum(float(M[j]) * Kc[j] for j in range(4))) <= 1.0 + 1e-14


def test_ros4_one_step_isomer(mech_dir):
    """One fixed ROS4 step on A <=> B moves the distance from equilibrium by
    exactly R(z) with z = -(kf + kr) h, and the error estimate is E(z) d0."""
    kf, shift = 2.0e5, 0.7
    M = O.Mech(_write(mechs.isomer_pair(kf, shift), mech_dir, "iso_r4"))
    kr = kf / math.exp(shift)
    yeq = kr / (kf + kr)
    _, gam, A, C, Mw, E = _tab_fractions(O.ROS4)
    for h in [1e-7, 3e-6, 1e-4, 1e-2]:
        y0 = np.array([1200.0, 0.9, 0.1])
        yn, err = M.step(1e5, y0, h, O.ROS4)
        R, Er = _ros_linear(gam, A, C, Mw, E, Fraction(-(kf + kr) * h))
        d0 = y0[1] - yeq
        assert yn[0] == y0[0]
        assert abs((yn[1] - yeq) - float(R) * d0) <= 1e-13 * abs(d0)
        assert abs(err[1] - float(Er) * d0) <= 1e-13 * abs(d0)


def test_ros4_convergence_order_termolecular(mech_dir):
    """Fixed-step ROS4 on 3A -> 3B (closed form C_A = C_A0 / sqrt(1 + 6 k
    C_A0^2 t)): the main solution converges as h^4, the embedded one as h^3."""
    k = 1.0e2
    mech = mechs.termolecular_isomer(k)
    M = O.Mech(_write(mech, mech_dir, "ter_r4"))
    T, p = 1000.0, 1.0e5
    y0 = np.array([T, 1.0, 0.0])
    C0 = p / (R_GAS * T)
    rho = p * mech.W[0] / (R_GAS * T)
    t_end = 2.0 / (k * C0 * C0)
    exact = C0 / math.sqrt(1 + 6 * k * C0 * C0 * t_end) * mech.W[0] / rho
    em, ee = [], []
    for N in [8, 16, 32, 64, 128]:
        h = t_end / N
        y, ye = y0.copy(), y0.copy()
        for _ in range(N):
            y, _ = M.step(p, y, h, O.ROS4)
            yn, e = M.step(p, ye, h, O.ROS4)
            ye = yn - e
        em.append(abs(y[1] - exact))
        ee.append(abs(ye[1] - exact))
    sm = [math.log2(em[i] / em[i + 1]) for i in range(4)]
    se = [math.log2(ee[i] / ee[i + 1]) for i in range(4)]
    assert abs(sm[-1] - 4.0) < 0.15 and abs(sm[-2] - 4.0) < 0.15, sm
    assert abs(se[-1] - 3.0) < 0.1 and abs(se[-2] - 3.0) < 0.15, se


def test_ros4_adaptive_closed_form_and_radau(mech_dir):
    """Adaptive ROS4 on the isomer pair meets the closed form within ten
    times the tolerance, and on 9-species cells agrees with Rodas3 within the
    same bound (two different schemes of the same accuracy target)."""
    kf, shift = 2.0e5, 0.7
    M = O.Mech(_write(mechs.isomer_pair(kf, shift), mech_dir, "iso2_r4"))
    kr = kf / math.exp(shift)
    yeq = kr / (kf + kr)
    phi = np.array([[1100.0, 1e5, 0.95, 0.05], [900.0, 1e5, 0.0, 1.0]])
    for dt in [1e-6, 1e-5, 1e-4]:
        out, h, na, nr, st = M.integrate(phi, dt, scheme=O.ROS4)
        assert (st == 0).all()
        ya = yeq + (phi[:, 2] - yeq) * math.exp(-(kf + kr) * dt)
        assert np.all(np.abs(out[:, 2] - ya) <= 10 * (1e-10 + 1e-6 * np.abs(ya)))
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", mech_dir, n_cells=64)
    T9 = O.Mech(path)
    a = T9.integrate(phi, wl.dt, scheme=O.ROS4, n_threads=4)
    b = T9.integrate(phi, wl.dt, scheme=O.RODAS3, n_threads=4)
    assert (a[4] == 0).all() and (b[4] == 0).all()
    tol = 1e-10 + 1e-6 * np.abs(b[0][:, 2:])
    assert np.all(np.abs(a[0][:, 2:] - b[0][:, 2:]) <= 10 * tol)
    assert np.all(np.abs(a[0][:, 0] - b[0][:, 0]) <= 10 * 1e-6 * b[0][:, 0])
    with pytest.raises(ValueError):
        T9.integrate(phi[:2], wl.dt, scheme=7)


# ------------------------------------- forward-difference Jacobian (NEXT-3) ---
# The integrator's FD mode stands for the conventional finite-difference
# Jacobian that the paper's analytical one replaces (Introduction; Fig. 2).

def test_jac_fd_isomer_closed_form(mech_dir):
    """A <=> B isomers at constant T: f is linear in Y, so forward
    differences reproduce the closed-form Jacobian (J_AA = -kf, J_AB = kr,
    J_BA = kf, J_BB = -kr, no T coupling) up to rounding over the increment."""
    kf, shift = 2.0e5, 0.7
    M = O.Mech(_write(mechs.isomer_pair(kf, shift), mech_dir, "iso_fd"))
    kr = kf / math.exp(shift)
    # the second state's f is dominated by kr Y_B ~ 1e5, whose rounding over
    # the 3e-11 increment of Y_A leaves ~1e-6 relative error in column A
    for y, rel in ((np.array([1200.0, 0.9, 0.1]), 1e-7), (np.array([800.0, 1e-12, 1.0 - 1e-12]), 1e-5)):
        J = M.jac_fd(1e5, y)
        exact = np.array([[0.0, 0.0, 0.0], [0.0, -kf, kr], [0.0, kf, -kr]])
        assert np.abs(J - exact).max() <= rel * kf, J


@pytest.mark.parametrize("name", ["tiny9_1024", "spray54_262144"])
def test_jac_fd_approximates_analytical(name, mech_dir):
    """On real states the FD Jacobian approximates the analytical one in the
    scaled form diag(1/s) J diag(s): on the 9-species cells every entry within
    1e-5 of its row's largest, on the 54-species cells at least 99.5% of the
    entries within 1e-4 of it. The rest are the columns of trace species
    (Y ~ 1e-12) on cold cells, where the increment sqrt(u 1e-5) ~ 3e-11 is
    far larger than Y and the quadratic terms of the rates spoil the forward
    difference: the inaccuracy the analytical Jacobian removes."""
    wl, mech, path, phi = synth.workload_inputs(name, mech_dir, n_cells=512)
    M = O.Mech(path)
    for c in synth.sample_indices(512, 8, 3):
        y = np.concatenate([[phi[c, 0]], phi[c, 2:]])
        Ja, Jf = M.jac(phi[c, 1], y), M.jac_fd(phi[c, 1], y)
        s = np.maximum(np.abs(y), [1.0] + [1e-8] * (len(y) - 1))
        A, B = Ja * s[None, :] / s[:, None], Jf * s[None, :] / s[:, None]
        rowmax = np.abs(A).max(axis=1, keepdims=True)
        r = np.where(rowmax > 0, np.abs(A - B) / np.where(rowmax > 0, rowmax, 1.0), 0.0)
        if mech.n_species == 9:
            assert r.max() <= 1e-5, c
        else:
            assert (r > 1e-4).mean() <= 5e-3 and np.percentile(r, 99) <= 1e-4, c


def test_integration_fd_jacobian_matches_analytical(mech_dir):
    """The integration with the FD Jacobian reaches the analytical run's
    states within ten times the tolerance (both approximate the same exact
    solution to it); an unknown Jacobian mode is rejected."""
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", mech_dir, n_cells=128)
    M = O.Mech(path)
    a = M.integrate(phi, wl.dt, n_threads=4)
    b = M.integrate(phi, wl.dt, n_threads=4, jacobian=O.JAC_FD)
    assert (a[4] == 0).all() and (b[4] == 0).all()
    tol = 1e-10 + 1e-6 * np.abs(a[0][:, 2:])
    assert np.all(np.abs(b[0][:, 2:] - a[0][:, 2:]) <= 10 * tol)
    assert np.all(np.abs(b[0][:, 0] - a[0][:, 0]) <= 10 * 1e-6 * a[0][:, 0])
    with pytest.raises(ValueError):
        M.integrate(phi[:2], wl.dt, jacobian=3)


# ------------------------------------------ bath gas dropped (NEXT-4) ---
# pyJac's state convention: the last species (the bath gas) is not
# integrated; its mass fraction is 1 - the sum of the others, n = Ns.

def test_no_bath_isomer_closed_form(mech_dir):
    """A <=> B with B the bath gas: y = (T, Y_A), f_A = -(kf + kr) Y_A + kr
    because Y_B = 1 - Y_A, so the reduced Jacobian is [[0, 0], [0, -(kf +
    kr)]]; the integration relaxes Y_A to equilibrium as the exponential."""
    kf, shift = 2.0e5, 0.7
    M = O.Mech(_write(mechs.isomer_pair(kf, shift), mech_dir, "iso_nb"))
    kr = kf / math.exp(shift)
    y = np.array([1200.0, 0.9])
    f = M.state_rhs(1e5, y, O.STATE_NO_BATH)
    J = M.state_jac(1e5, y, O.STATE_NO_BATH)
    assert abs(f[1] - (-(kf + kr) * 0.9 + kr)) <= 1e-12 * kf
    assert abs(f[0]) <= 1e-9 * kf
    assert np.abs(J - np.array([[0.0, 0.0], [0.0, -(kf + kr)]])).max() <= 1e-9 * kf
    yeq = kr / (kf + kr)
    phi = np.array([[1100.0, 1e5, 0.95, 0.05], [900.0, 1e5, 0.0, 1.0]])
    for dt in [1e-6, 1e-5, 1e-4]:
        out, h, na, nr, st = M.integrate(phi, dt, state=O.STATE_NO_BATH)
        assert (st == 0).all()
        ya = yeq + (phi[:, 2] - yeq) * math.exp(-(kf + kr) * dt)
        assert np.all(np.abs(out[:, 2] - ya) <= 10 * (1e-10 + 1e-6 * np.abs(ya)))
        assert np.all(out[:, 3] == 1.0 - out[:, 2])


@pytest.mark.parametrize("name", ["tiny9_1024", "spray54_262144"])
def test_no_bath_jacobian_vs_finite_differences(name, mech_dir):
    """The reduced Jacobian (the full one's columns minus its last column, by
    the chain rule through Y_Ns = 1 - sum Y_j) against central differences of
    the reduced right-hand side itself, in the scaled form of R22."""
    wl, mech, path, phi = synth.workload_inputs(name, mech_dir, n_cells=512)
    M = O.Mech(path)
    for c in synth.sample_indices(512, 8, 5):
        y = np.concatenate([[phi[c, 0]], phi[c, 2:-1]])      # without the last species
        p = phi[c, 1]
        n = len(y)
        s = np.abs(y).copy()
        s[0] = max(s[0], 1.0)
        s[1:] = np.maximum(s[1:], 1e-8)
        J = M.state_jac(p, y, O.STATE_NO_BATH)
        Jfd = np.zeros_like(J)
        for j in range(n):
            d = 1e-6 * s[j]
            yp, ym = y.copy(), y.copy()
            yp[j] += d
            ym[j] -= d
            Jfd[:, j] = (M.state_rhs(p, yp, O.STATE_NO_BATH) - M.state_rhs(p, ym, O.STATE_NO_BATH)) / (2 * d)
        Ja = J * s[None, :] / s[:, None]
        Jf = Jfd * s[None, :] / s[:, None]
        rowmax = np.abs(Ja).max(axis=1, keepdims=True)
        assert not (np.abs(Ja - Jf) > 1e-6 * np.abs(Jf) + 1e-9 * rowmax).any(), c


def test_no_bath_integration_matches_full_state(mech_dir):
    """Dropping the bath gas integrates the same ODE: the states agree with
    the full-state integration within ten times the tolerance, the mass
    fractions sum to one to rounding, and the input's last mass fraction is
    not read."""
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", mech_dir, n_cells=128)
    M = O.Mech(path)
    a = M.integrate(phi, wl.dt, n_threads=4)
    b = M.integrate(phi, wl.dt, n_threads=4, state=O.STATE_NO_BATH)
    assert (a[4] == 0).all() and (b[4] == 0).all()
    tol = 1e-10 + 1e-6 * np.abs(a[0][:, 2:])
    assert np.all(np.abs(b[0][:, 2:] - a[0][:, 2:]) <= 10 * tol)
    assert np.all(np.abs(b[0][:, 0] - a[0][:, 0]) <= 10 * 1e-6 * a[0][:, 0])
    assert np.abs(b[0][:, 2:].sum(axis=1) - 1.0).max() <= 4e-16
    junk = phi.copy()
    junk[:, -1] = 123.0
    c = M.integrate(junk, wl.dt, n_threads=4, state=O.STATE_NO_BATH)
    assert np.array_equal(c[0], b[0]) and np.array_equal(c[2], b[2])
    with pytest.raises(ValueError):
        M.integrate(phi[:2], wl.dt, state=2)


# ------------------------------------------- evaluation counters (a8) ---
# njac counts step starts (the first state and every state an accepted step
# leads to that the integration continues from), nfev adds the new-point
# stages of every attempt whose LU succeeded (two for Rodas3: stages 3 and 4;
# two for ROS4, whose stage 4 reuses stage 3's point) and the n evaluations
# of a forward-difference Jacobian. Pinned here by the step sequence alone.

def test_eval_counts_follow_the_step_sequence(mech_dir):
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", mech_dir, n_cells=64)
    M = O.Mech(path)
    n = mech.n_species + 1
    for scheme in (O.RODAS3, O.ROS4):
        out, h, na, nr, st, nj, nf = M.integrate(phi, wl.dt, scheme=scheme, counts=True)
        assert (st == 0).all() and (na >= 1).all()
        assert np.array_equal(nj, na)                      # one Jacobian per accepted step's start state
        assert np.array_equal(nf, nj + 2 * (na + nr))
        # the same run without counting gives the same results
        out2, h2, na2, nr2, st2 = M.integrate(phi, wl.dt, scheme=scheme)
        assert np.array_equal(out, out2) and np.array_equal(na, na2)
    out, h, na, nr, st, nj, nf = M.integrate(phi, wl.dt, jacobian=O.JAC_FD, counts=True)
    assert np.array_equal(nj, na) and np.array_equal(nf, nj * (1 + n) + 2 * (na + nr))
    out, h, na, nr, st, nj, nf = M.integrate(phi, wl.dt, jacobian=O.JAC_FD, state=O.STATE_NO_BATH, counts=True)
    assert np.array_equal(nf, nj * (1 + (n - 1)) + 2 * (na + nr))


def test_eval_counts_at_failures(mech_dir):
    wl, mech, path, phi = synth.workload_inputs("tiny9_1024", mech_dir, n_cells=8)
    M = O.Mech(path)
    # step underflow: every attempt from the first state, one Jacobian
    out, h, na, nr, st, nj, nf = M.integrate(phi, wl.dt, rtol=1e-30, atol=1e-300, counts=True)
    assert (st == 2).all() and (na == 0).all() and (nj == 1).all()
    assert np.array_equal(nf, 1 + 2 * nr)
    # one attempt allowed: one start; a cell that needs more stops before
    # evaluating the next state's Jacobian
    out, h, na, nr, st, nj, nf = M.integrate(phi, wl.dt, max_steps=1, counts=True)
    assert (na + nr == 1).all() and (nj == 1).all() and (nf == 3).all()
    # a non-finite input is not integrated
    bad = phi.copy()
    bad[:, 3] = np.nan
    out, h, na, nr, st, nj, nf = M.integrate(bad, wl.dt, counts=True)
    assert (st == 3).all() and (nj == 0).all() and (nf == 0).all()
