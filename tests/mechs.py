"""Small hand-built mechanisms with closed-form behaviour, for pinning the
oracle (and the GPU library) against mathematics rather than against itself."""
import numpy as np

from paper_2112_05834_amd import synth

R_GAS = 8.314462618
P_ATM = 101325.0


def _nasa(cp0=3.5, dcp=0.0, h=0.0, s=20.0):
    return synth.nasa_from_draws(cp0, dcp, h, s)


def _mech(comps, nasa, reactions, names=None):
    elem = np.array([list(c) + [0] * (4 - len(c)) for c in comps], dtype=np.int64)
    W = elem @ np.array(synth.ELEMENT_WEIGHTS)
    names = names or ["S%d" % i for i in range(len(comps))]
    nasa = np.array(nasa)
    return synth.Mechanism(names=names, W=W, elem=elem, nasa_lo=nasa.copy(), nasa_hi=nasa.copy(),
                           reactions=reactions)


def isomer_pair(kf_A=2.0e5, a7_shift=0.7, reversible=True):
    """A <=> B with equal W and equal NASA coefficients except a7: dH = 0 so T
    stays constant, Kc = exp(a7_B - a7_A), and Y_A relaxes exponentially with
    rate kf + kr."""
    nA = _nasa(h=-1000.0, s=25.0)
    nB = nA.copy()
    nB[6] += a7_shift
    # A and B must have equal W: give them the same composition
    rx = [synth.Reaction(synth.ELEMENTARY, reversible, [(0, 1)], [(1, 1)], kf_A, 0.0, 0.0)]
    return _mech([(1, 1, 1, 0), (1, 1, 1, 0)], [nA, nB], rx, names=["A", "B"])


def bimolecular_abcd(k=3.0e3):
    """A + B -> C + D, irreversible, all four species with identical NASA
    coefficients (dH = 0, T constant) and W_A + W_B = W_C + W_D, so moles and
    density are conserved and C_A = C_A0 / (1 + k C_A0 t) when C_A0 = C_B0."""
    n = _nasa(cp0=4.0, dcp=1.0, h=-500.0, s=22.0)
    rx = [synth.Reaction(synth.ELEMENTARY, False, [(0, 1), (1, 1)], [(2, 1), (3, 1)], k, 0.0, 0.0)]
    return _mech([(1, 1, 0, 0), (0, 0, 1, 0), (1, 0, 1, 0), (0, 1, 0, 0)], [n, n, n, n], rx,
                 names=["A", "B", "C", "D"])


def termolecular_isomer(k=1.0e2):
    """3 A -> 3 B, irreversible, third order in A, with A and B isomers of
    identical NASA coefficients: moles, density and T are constant, so
    dC_A/dt = -3 k C_A^3 and C_A = C_A0 / sqrt(1 + 6 k C_A0^2 t). (A
    second-order reaction would not do: Rodas3's first stage is the linearly
    implicit trapezoidal rule, which is exact for Riccati equations.)"""
    n = _nasa(cp0=4.0, dcp=1.0, h=-500.0, s=22.0)
    rx = [synth.Reaction(synth.ELEMENTARY, False, [(0, 3)], [(1, 3)], k, 0.0, 0.0)]
    return _mech([(1, 1, 1, 0), (1, 1, 1, 0)], [n, n], rx, names=["A", "B"])


def isomer_cycle(a7_shifts=(0.0, 0.9, -0.4), kf=(5e5, 3e5, 8e5)):
    """Three isomers A, B, C in the cycle A<=>B, B<=>C, A<=>C with equal h:
    the equilibrium mole (= mass) fractions are proportional to exp(a7_i)."""
    base = _nasa(h=-2000.0, s=24.0)
    n = []
    for d in a7_shifts:
        x = base.copy()
        x[6] += d
        n.append(x)
    rx = [synth.Reaction(synth.ELEMENTARY, True, [(0, 1)], [(1, 1)], kf[0], 0.0, 0.0),
          synth.Reaction(synth.ELEMENTARY, True, [(1, 1)], [(2, 1)], kf[1], 0.0, 0.0),
          synth.Reaction(synth.ELEMENTARY, True, [(0, 1)], [(2, 1)], kf[2], 0.0, 0.0)]
    return _mech([(1, 1, 1, 0)] * 3, n, rx, names=["A", "B", "C"])


def dissociation(kf=1e8):
    """A <=> B + B with h_A = 2 h_B at every T (so T stays constant) and
    different entropies: C_B^2 / C_A = Kc at equilibrium, with Kc carrying the
    (p_atm / RT)^1 factor."""
    nB = _nasa(cp0=2.5, dcp=0.0, h=1000.0, s=20.0)
    nA = synth.nasa_from_draws(5.0, 0.0, 2000.0, 30.0)
    rx = [synth.Reaction(synth.ELEMENTARY, True, [(0, 1)], [(1, 2)], kf, 0.0, 0.0)]
    return _mech([(0, 2, 0, 0), (0, 1, 0, 0)], [nA, nB], rx, names=["A", "B"])


def third_body_unit(A=1.0e2):
    """A + B + M -> C + M with all efficiencies 1 (no 'eff' entries):
    [M] = sum C_i = p / (RT)."""
    n = [_nasa(h=-100.0 * i) for i in range(4)]
    rx = [synth.Reaction(synth.THIRD_BODY, False, [(0, 1), (1, 1)], [(2, 1)], A, 0.0, 0.0, eff=[])]
    return _mech([(1, 0, 0, 0), (0, 0, 1, 0), (1, 0, 1, 0), (0, 0, 0, 2)], n, rx)


def troe_lindemann(A=1.0e7, A0=1.0e4):
    """A + B (+M) -> C with Troe a = 1, T1 huge, no T2: Fcent = 1, so F = 1 and
    k = k_inf Pr / (1 + Pr) (Lindemann)."""
    n = [_nasa(h=-100.0 * i) for i in range(4)]
    rx = [synth.Reaction(synth.TROE, False, [(0, 1), (1, 1)], [(2, 1)], A, 0.0, 0.0, eff=[],
                         troe=(A0, 0.0, 0.0, 1.0, 100.0, 1e30, 0.0, 0.0))]
    return _mech([(1, 0, 0, 0), (0, 0, 1, 0), (1, 0, 1, 0), (0, 0, 0, 2)], n, rx)


def troe_mix(seed=5):
    """A few reversible third-body and Troe reactions with non-unit
    efficiencies and Troe parameters in the falloff region, for derivative
    checks of the falloff chain rule."""
    rng = np.random.Generator(np.random.PCG64(seed))
    comps = [(1, 0, 0, 0), (0, 0, 1, 0), (1, 0, 1, 0), (2, 0, 1, 0), (2, 0, 0, 0), (0, 0, 0, 2)]
    nasa = [_nasa(cp0=2.5 + sum(c) - 1, dcp=0.5 * (sum(c) - 1), h=rng.uniform(-2e4, 2e4),
                  s=15 + 3 * sum(c)) for c in comps]
    rx = [
        synth.Reaction(synth.TROE, True, [(0, 1), (2, 1)], [(3, 1)], 3e8 * 1e-6, 0.3, 2000.0,
                       eff=[(4, 2.5), (5, 0.7)], troe=(2e16 * 1e-12, -1.2, 500.0, 0.6, 150.0, 2500.0, 4000.0, 1.0)),
        synth.Reaction(synth.TROE, True, [(0, 1), (0, 1)], [(4, 1)], 1e9 * 1e-6, 0.0, 0.0,
                       eff=[(3, 6.0)], troe=(1e18 * 1e-12, -1.0, 0.0, 0.4, 300.0, 1500.0, 0.0, 0.0)),
        synth.Reaction(synth.THIRD_BODY, True, [(0, 1), (1, 1)], [(2, 1)], 5e17 * 1e-12, -1.0, 0.0,
                       eff=[(3, 12.0), (4, 2.0)]),
        synth.Reaction(synth.ELEMENTARY, True, [(0, 1), (3, 1)], [(4, 1), (1, 1)], 2e13 * 1e-6, 0.0, 3e4),
    ]
    return _mech(comps, nasa, rx)


def third_body_efficiencies(A=1.0e2, alpha_zero=2, alpha_three=3):
    """A + B + M -> C + M (species 0..3) with efficiency 0 for species
    alpha_zero and 3 for species alpha_three, all others 1:
    [M] = p/(RT) - C_k + 2 C_k' exactly."""
    n = [_nasa(h=-100.0 * i) for i in range(4)]
    rx = [synth.Reaction(synth.THIRD_BODY, False, [(0, 1), (1, 1)], [(2, 1)], A, 0.0, 0.0,
                         eff=[(alpha_zero, 0.0), (alpha_three, 3.0)])]
    return _mech([(1, 0, 0, 0), (0, 0, 1, 0), (1, 0, 1, 0), (0, 0, 0, 2)], n, rx)


def troe_general(A=3.0e6, b=0.7, Ea=2.2e4, A0=5.0e3, b0=-1.3, Ea0=9.0e3,
                 a=0.62, T3=170.0, T1=1900.0, T2=4300.0, eff=((2, 0.0), (3, 3.0))):
    """A + B (+M) -> C with every Troe parameter active (a, T3, T1, T2), both
    rate constants of modified-Arrhenius form with b != 0 and Ea != 0, and
    non-unit efficiencies; irreversible, so q = k_inf Pr/(1+Pr) F C_A C_B."""
    n = [_nasa(h=-100.0 * i) for i in range(4)]
    rx = [synth.Reaction(synth.TROE, False, [(0, 1), (1, 1)], [(2, 1)], A, b, Ea, eff=list(eff),
                         troe=(A0, b0, Ea0, a, T3, T1, T2, 1.0))]
    return _mech([(1, 0, 0, 0), (0, 0, 1, 0), (1, 0, 1, 0), (0, 0, 0, 2)], n, rx)


def arrhenius_isomer(A=4.0e9, b=1.7, Ea=8.5e4, a7_shift=0.45):
    """A <=> B isomers (equal W, equal NASA coefficients except a7) with a
    modified-Arrhenius forward rate: ln kf = ln A + b ln T - (Ea/R)/T and,
    since Kc = exp(a7_B - a7_A) does not depend on T, ln kr = ln kf - a7_shift."""
    nA = _nasa(h=-1000.0, s=25.0)
    nB = nA.copy()
    nB[6] += a7_shift
    rx = [synth.Reaction(synth.ELEMENTARY, True, [(0, 1)], [(1, 1)], A, b, Ea)]
    return _mech([(1, 1, 1, 0), (1, 1, 1, 0)], [nA, nB], rx, names=["A", "B"])
