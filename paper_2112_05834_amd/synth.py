"""Seeded synthetic inputs: kinetic mechanisms and cell states.

The paper's own mechanisms (a 54-species / 269-reaction n-dodecane model and
GRI-3.0) and its CFD fields are not available, so every workload here is drawn
from a seeded generator with the same shape: species count, reaction count,
third-body and Troe falloff counts, pressures, temperature and composition
distributions.

This module only draws random numbers and writes them out. It evaluates no
thermodynamics, no rate constant and no integration: the thermo polynomial
coefficients are constructed in closed form from drawn heat capacities,
formation enthalpies and entropies. Both the CPU oracle and the GPU library
parse the text file written by :func:`write_mech`, each with its own parser.

Mechanism file format (whitespace separated tokens, ``#`` starts a comment)::

    chemmech 1
    elements <Ne>
    <name> <atomic weight kg/mol>                       (Ne lines)
    species <Ns>
    <name> <W kg/mol> <Tlow> <Tmid> <Thigh> <count_e0> ... <count_e(Ne-1)>
    <a1..a7 for T < Tmid>
    <a1..a7 for T >= Tmid>                              (Ns blocks)
    reactions <Nr>
    reaction <type> <reversible> <n_reac> (<sp> <order>)* <n_prod> (<sp> <order>)* <A> <b> <Ea>
    [eff <k> (<sp> <alpha>)*]                           (type 1 and 2)
    [troe <A0> <b0> <Ea0> <a> <T3> <T1> <T2> <has_T2>]  (type 2)
    end

Types: 0 elementary, 1 third body (+M), 2 Troe falloff (+M). Units are SI
with mol: A in (m^3/mol)^(m-1)/s for a reaction of order m (third body
counted), Ea in J/mol, W in kg/mol.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

ELEMENT_NAMES = ("E0", "E1", "E2", "E3")
ELEMENT_WEIGHTS = (1.008e-3, 12.011e-3, 15.999e-3, 14.007e-3)  # kg/mol

T_LOW, T_MID, T_HIGH = 200.0, 1000.0, 6000.0

ELEMENTARY, THIRD_BODY, TROE = 0, 1, 2


@dataclasses.dataclass
class Reaction:
    rtype: int
    reversible: bool
    reac: List[Tuple[int, int]]          # (species, order)
    prod: List[Tuple[int, int]]
    A: float
    b: float
    Ea: float
    eff: List[Tuple[int, float]] = dataclasses.field(default_factory=list)
    troe: Optional[Tuple[float, ...]] = None   # A0 b0 Ea0 a T3 T1 T2 has_T2


@dataclasses.dataclass
class Mechanism:
    names: List[str]
    W: np.ndarray                 # [Ns] kg/mol
    elem: np.ndarray              # [Ns, Ne] atom counts
    nasa_lo: np.ndarray           # [Ns, 7]
    nasa_hi: np.ndarray           # [Ns, 7]
    reactions: List[Reaction]
    t_ranges: np.ndarray = None   # [Ns, 3]
    inert: int = -1
    fuel: int = -1
    oxidiser: int = -1
    products: List[int] = dataclasses.field(default_factory=list)
    radicals: List[int] = dataclasses.field(default_factory=list)

    @property
    def n_species(self) -> int:
        return len(self.names)

    @property
    def n_reactions(self) -> int:
        return len(self.reactions)

    def type_counts(self) -> Tuple[int, int, int]:
        t = [r.rtype for r in self.reactions]
        return t.count(ELEMENTARY), t.count(THIRD_BODY), t.count(TROE)


# --------------------------------------------------------------------------
# file writer
# --------------------------------------------------------------------------

def _g(x: float) -> str:
    return "%.17g" % float(x)


def write_mech(mech: Mechanism, path: str) -> str:
    """Write ``mech`` in the text format above; returns ``path``."""
    ns = mech.n_species
    tr = mech.t_ranges
    if tr is None:
        tr = np.tile([T_LOW, T_MID, T_HIGH], (ns, 1))
    lines = ["chemmech 1", "elements %d" % len(ELEMENT_NAMES)]
    for n, w in zip(ELEMENT_NAMES, ELEMENT_WEIGHTS):
        lines.append("%s %s" % (n, _g(w)))
    lines.append("species %d" % ns)
    for i in range(ns):
        lines.append(" ".join([mech.names[i], _g(mech.W[i]), _g(tr[i, 0]), _g(tr[i, 1]), _g(tr[i, 2])]
                              + [str(int(c)) for c in mech.elem[i]]))
        lines.append(" ".join(_g(a) for a in mech.nasa_lo[i]))
        lines.append(" ".join(_g(a) for a in mech.nasa_hi[i]))
    lines.append("reactions %d" % mech.n_reactions)
    for r in mech.reactions:
        tok = ["reaction", str(r.rtype), "1" if r.reversible else "0", str(len(r.reac))]
        for s, o in r.reac:
            tok += [str(s), str(o)]
        tok.append(str(len(r.prod)))
        for s, o in r.prod:
            tok += [str(s), str(o)]
        tok += [_g(r.A), _g(r.b), _g(r.Ea)]
        lines.append(" ".join(tok))
        if r.rtype in (THIRD_BODY, TROE):
            lines.append(" ".join(["eff", str(len(r.eff))] + [f"{s} {_g(a)}" for s, a in r.eff]))
        if r.rtype == TROE:
            lines.append(" ".join(["troe"] + [_g(v) for v in r.troe[:7]] + [str(int(r.troe[7]))]))
    lines.append("end")
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    os.replace(tmp, path)
    return path


# --------------------------------------------------------------------------
# thermo coefficients in closed form from drawn quantities
# --------------------------------------------------------------------------

def nasa_from_draws(cp0: float, dcp: float, h_const: float, s298: float) -> np.ndarray:
    """NASA-7 coefficients of a heat capacity cp/R(T) = cp0 + dcp*s(x),
    x = (T-200)/5800, s(x) = 3x^2 - 2x^3 (monotone on [200, 6000] K), with
    enthalpy constant a6 = h_const [K] and the entropy constant chosen so
    that s/R(298.15 K) = s298."""
    al = 1.0 / (T_HIGH - T_LOW)
    be = -T_LOW / (T_HIGH - T_LOW)
    a1 = cp0 + dcp * (3 * be * be - 2 * be ** 3)
    a2 = dcp * (6 * al * be - 6 * al * be * be)
    a3 = dcp * (3 * al * al - 6 * al * al * be)
    a4 = dcp * (-2 * al ** 3)
    a5 = 0.0
    t = 298.15
    s_poly = a1 * math.log(t) + a2 * t + a3 * t * t / 2 + a4 * t ** 3 / 3 + a5 * t ** 4 / 4
    a7 = s298 - s_poly
    return np.array([a1, a2, a3, a4, a5, h_const, a7], dtype=np.float64)


# --------------------------------------------------------------------------
# species and reaction topology
# --------------------------------------------------------------------------

def _composition_pool(elems: Sequence[int], total: int) -> List[Tuple[int, ...]]:
    out = []

    def rec(prefix, left, k):
        if k == len(elems) - 1:
            out.append(tuple(prefix + [left]))
            return
        for c in range(left, -1, -1):
            rec(prefix + [c], left - c, k + 1)

    rec([], total, 0)
    return out


def _species_set(rng: np.random.Generator, n_noninert: int, elems: Sequence[int]):
    chosen: List[Tuple[int, ...]] = []
    ox = tuple(2 if e == 2 else 0 for e in elems)
    chosen.append(ox)
    total = 1
    while len(chosen) < n_noninert:
        level = [c for c in _composition_pool(elems, total) if c not in chosen]
        rng.shuffle(level)
        need = n_noninert - len(chosen)
        chosen += level[:need]
        total += 1
    comps = []
    for c in chosen:
        full = [0, 0, 0, 0]
        for e, k in zip(elems, c):
            full[e] = k
        comps.append(tuple(full))
    comps.sort(key=lambda v: (sum(v), v))
    return comps


def _is_radical(comp: Tuple[int, ...]) -> bool:
    if sum(comp) == 1:
        return True
    return comp[0] % 2 == 1


def _species_name(comp: Tuple[int, ...]) -> str:
    s = ""
    for e, k in enumerate(comp):
        if k:
            s += "ABCD"[e] + (str(k) if k > 1 else "")
    return s


def generate_mechanism(n_species: int, n_reactions: int, n_third_body: int, n_troe: int,
                       seed: int, ea_by_class: bool = False) -> Mechanism:
    """Seeded synthetic mechanism with ``n_species`` species (one inert E3_2
    collision partner), ``n_reactions`` reversible reactions of which
    ``n_third_body`` are third-body and ``n_troe`` Troe falloff reactions
    (disjoint sets), all element balanced.

    Arrhenius draws: A' log-uniform in [1e6, 1e14] (CGS magnitude of the rate
    constant at 1000 K), b ~ U[-1, 2]. Activation energies are Ea ~ U[0, 2e5]
    J/mol, or with ``ea_by_class`` U[1.5e5, 2.5e5] for reactions without a
    radical reactant and U[0, 1e5] otherwise, so that unburnt mixtures stay
    slow while radical chemistry is fast and stiff."""
    rng = np.random.Generator(np.random.PCG64(seed))
    elems = (0, 2) if n_species <= 12 else (0, 1, 2)
    comps = _species_set(rng, n_species - 1, elems)
    comps.append((0, 0, 0, 2))          # inert, last
    ns = len(comps)
    inert = ns - 1
    elem = np.array(comps, dtype=np.int64)
    W = elem @ np.array(ELEMENT_WEIGHTS)
    names = [_species_name(c) for c in comps]
    radicals = [i for i in range(ns - 1) if _is_radical(comps[i])]
    stable = [i for i in range(ns - 1) if i not in radicals]
    ox = comps.index(tuple(2 if e == 2 else 0 for e in range(4)))
    fuel_cands = [i for i in stable if comps[i][2] == 0 and i != ox]
    fuel = max(fuel_cands, key=lambda i: (comps[i][0] + comps[i][1], W[i]))
    products = [i for i in stable if i not in (fuel, ox)]

    # thermo draws
    nasa = np.zeros((ns, 7))
    for i, c in enumerate(comps):
        atoms = sum(c)
        if atoms == 1:
            cp0, dcp = 2.5, 0.0
        else:
            cp0 = 2.5 + (atoms - 1) + rng.uniform(0.0, 0.5)
            dcp = (atoms - 1) * rng.uniform(1.0, 1.8)
        if i == inert:
            hf = 0.0
        elif i in radicals:
            hf = rng.uniform(0.0, 3.0e4)
        else:
            hf = rng.uniform(-3.0e4, 0.0)
        s298 = 15.0 + 3.0 * atoms + rng.normal(0.0, 1.0)
        nasa[i] = nasa_from_draws(cp0, dcp, hf, s298)

    # balanced candidates over non-inert species
    noninert = list(range(ns - 1))
    pairs: Dict[Tuple[int, ...], List[Tuple[int, int]]] = {}
    for ia, a in enumerate(noninert):
        for b in noninert[ia:]:
            key = tuple(elem[a] + elem[b])
            pairs.setdefault(key, []).append((a, b))
    recomb = []   # (a, b, c): a + b -> c
    for c in noninert:
        for (a, b) in pairs.get(tuple(elem[c]), []):
            recomb.append((a, b, c))
    keys_multi = [k for k, v in pairs.items() if len(v) >= 2]

    def exch_candidates_with(s):
        out = []
        for k in keys_multi:
            v = pairs[k]
            for p1 in v:
                if s not in p1:
                    continue
                for p2 in v:
                    if p2 != p1 and not (set(p1) & set(p2)):
                        out.append((p1, p2))
        return out

    n_exch = n_reactions - n_third_body - n_troe
    chosen_keys = set()
    exch: List[Tuple[Tuple[int, int], Tuple[int, int]]] = []
    rec_sel: List[Tuple[int, int, int]] = []

    def rkey(p1, p2):
        return frozenset([tuple(sorted(p1)), tuple(sorted(p2))])

    # coverage first: every non-inert species in at least one reaction
    covered = set()
    order = list(noninert)
    rng.shuffle(order)
    for s in order:
        if s in covered:
            continue
        cands = exch_candidates_with(s) if len(exch) < n_exch else []
        if cands:
            p1, p2 = cands[rng.integers(len(cands))]
            k = rkey(p1, p2)
            if k not in chosen_keys:
                chosen_keys.add(k)
                exch.append((p1, p2))
                covered |= set(p1) | set(p2)
                continue
        rc = [t for t in recomb if s in t and ("R",) + t not in chosen_keys]
        if rc and len(rec_sel) < n_third_body + n_troe:
            t = rc[rng.integers(len(rc))]
            chosen_keys.add(("R",) + t)
            rec_sel.append(t)
            covered |= set(t)
    if len(covered) < ns - 1:
        raise RuntimeError("mechanism seed %d: could not cover every species" % seed)
    # fill the remainder at random
    guard = 0
    while len(exch) < n_exch:
        guard += 1
        if guard > 200000:
            raise RuntimeError("mechanism seed %d: not enough exchange reactions" % seed)
        k = keys_multi[rng.integers(len(keys_multi))]
        v = pairs[k]
        i1, i2 = rng.integers(len(v)), rng.integers(len(v))
        p1, p2 = v[i1], v[i2]
        if i1 == i2 or set(p1) & set(p2):
            continue
        kk = rkey(p1, p2)
        if kk in chosen_keys:
            continue
        chosen_keys.add(kk)
        exch.append((p1, p2))
    guard = 0
    while len(rec_sel) < n_third_body + n_troe:
        guard += 1
        if guard > 200000:
            raise RuntimeError("mechanism seed %d: not enough recombination reactions" % seed)
        t = recomb[rng.integers(len(recomb))]
        if ("R",) + t in chosen_keys:
            continue
        chosen_keys.add(("R",) + t)
        rec_sel.append(t)

    def side(species):
        d: Dict[int, int] = {}
        for s in species:
            d[s] = d.get(s, 0) + 1
        return sorted(d.items())

    def hf_of(side_list):
        return sum(o * nasa[s, 5] for s, o in side_list)

    def rate_draw(order_m, reac):
        a_ref = 10.0 ** rng.uniform(6.0, 14.0)
        b = rng.uniform(-1.0, 2.0)
        if ea_by_class and not any(s in radicals for s, _ in reac):
            ea = rng.uniform(1.5e5, 2.5e5)     # molecule-molecule: slow initiation
        elif ea_by_class:
            ea = rng.uniform(0.0, 1.0e5)       # radical attack / recombination
        else:
            ea = rng.uniform(0.0, 2.0e5)
        a_cgs = a_ref / 1000.0 ** b
        return a_cgs * (1e-6) ** (order_m - 1), b, ea

    def eff_draw():
        k = int(rng.integers(0, 7))
        sp = rng.choice(ns, size=k, replace=False) if k else []
        return [(int(s), float(rng.uniform(0.3, 12.0))) for s in sorted(sp)]

    reactions: List[Reaction] = []
    specs = [("E", p1, p2) for p1, p2 in exch]
    troe_idx = set(rng.choice(len(rec_sel), size=n_troe, replace=False).tolist()) if n_troe else set()
    for j, (a, b, c) in enumerate(rec_sel):
        specs.append(("F" if j in troe_idx else "T", (a, b), (c,)))
    perm = rng.permutation(len(specs))
    for idx in perm:
        kind, lhs, rhs = specs[idx]
        reac, prod = side(lhs), side(rhs)
        if hf_of(prod) - hf_of(reac) > 0.0:      # orient exothermic as written
            reac, prod = prod, reac
        order_f = sum(o for _, o in reac)
        if kind == "E":
            A, bb, ea = rate_draw(order_f, reac)
            reactions.append(Reaction(ELEMENTARY, True, reac, prod, A, bb, ea))
        elif kind == "T":
            A, bb, ea = rate_draw(order_f + 1, reac)
            reactions.append(Reaction(THIRD_BODY, True, reac, prod, A, bb, ea, eff=eff_draw()))
        else:
            A, bb, ea = rate_draw(order_f, reac)
            a0_ref = 10.0 ** rng.uniform(12.0, 18.0)
            b0 = rng.uniform(-2.0, 0.5)
            ea0 = rng.uniform(0.0, 1.0e5)
            A0 = a0_ref / 1000.0 ** b0 * (1e-6) ** order_f
            ta = rng.uniform(0.3, 0.9)
            t3 = 10.0 ** rng.uniform(math.log10(50.0), math.log10(500.0))
            t1 = 10.0 ** rng.uniform(3.0, 4.0)
            has_t2 = bool(rng.uniform() < 0.5)
            t2 = 10.0 ** rng.uniform(3.0, 4.0) if has_t2 else 0.0
            reactions.append(Reaction(TROE, True, reac, prod, A, bb, ea, eff=eff_draw(),
                                      troe=(A0, b0, ea0, ta, t3, t1, t2, 1.0 if has_t2 else 0.0)))
    return Mechanism(names=names, W=W, elem=elem, nasa_lo=nasa.copy(), nasa_hi=nasa.copy(),
                     reactions=reactions, inert=inert, fuel=fuel, oxidiser=ox,
                     products=products, radicals=radicals)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

# (n_species, n_reactions, n_third_body, n_troe, mechanism seed, ea_by_class)
MECHS = {
    "tiny9": (9, 20, 4, 0, 9, False),
    "spray54": (54, 269, 40, 12, 54, True),
    "large160": (160, 800, 120, 40, 160, True),
}

P_ATM = 101325.0


@dataclasses.dataclass
class Workload:
    name: str
    mech: str
    n_cells: int
    pressure: float
    dt: float
    state_seed: int
    recipe: str           # "uniform" | "bimodal" | "heavytail" | "ambient"
    n_steps: int = 1


WORKLOADS = {
    "tiny9_1024": Workload("tiny9_1024", "tiny9", 1024, P_ATM, 1e-6, 101, "uniform"),
    "spray54_262144": Workload("spray54_262144", "spray54", 262144, 6.0e6, 1e-6, 102, "bimodal"),
    "spray54_heavytail_1048576": Workload("spray54_heavytail_1048576", "spray54", 1048576, 6.0e6,
                                          1e-6, 103, "heavytail", n_steps=10),
    "large160_524288": Workload("large160_524288", "large160", 524288, 4.0e6, 5e-7, 105, "bimodal"),
    "spray54_ambient_262144": Workload("spray54_ambient_262144", "spray54", 262144, 6.0e6, 1e-6, 102,
                                       "ambient"),
    "large160_ambient_524288": Workload("large160_ambient_524288", "large160", 524288, 4.0e6, 5e-7, 105,
                                        "ambient"),
}

# Weights of the elements in Bilger's coupling function, per mole of atoms:
# E0 is hydrogen-like (1/2), E1 carbon-like (2), E2 oxygen-like (-1), E3 the
# inert nitrogen-like element (0).
BILGER_COUPLING = (0.5, 2.0, -1.0, 0.0)


def bilger_streams(mech: Mechanism):
    """(coupling [Ne], y_fuel [Ns], y_ox [Ns]) for the mixture fraction of a
    synthetic mechanism: the fuel stream is the pure fuel species, the
    oxidiser stream the 0.23:0.77 oxidiser:inert mixture of the unburnt cells."""
    ns = mech.n_species
    yf = np.zeros(ns)
    yf[mech.fuel] = 1.0
    yo = np.zeros(ns)
    yo[mech.oxidiser] = 0.23
    yo[mech.inert] = 0.77
    return np.array(BILGER_COUPLING[:mech.elem.shape[1]]), yf, yo


def mech_cached(name: str, directory: str) -> Tuple[Mechanism, str]:
    """Generate the named mechanism and write it under ``directory``."""
    ns, nr, n3, nt, seed, by_class = MECHS[name]
    mech = generate_mechanism(ns, nr, n3, nt, seed, ea_by_class=by_class)
    os.makedirs(directory, exist_ok=True)
    path = os.path.join(directory, "%s_seed%d.mech" % (name, seed))
    write_mech(mech, path)
    return mech, path


def _unburnt(rng, mech: Mechanism, n: int) -> np.ndarray:
    ns = mech.n_species
    Y = np.full((n, ns), 1e-12)
    yf = rng.uniform(0.05, 0.3, size=n)
    Y[:, mech.fuel] = yf
    Y[:, mech.oxidiser] = 0.23 * (1 - yf)
    Y[:, mech.inert] = 0.77 * (1 - yf)
    return Y / Y.sum(axis=1, keepdims=True)


def _hot_templates(rng, mech: Mechanism, k: int) -> np.ndarray:
    ns = mech.n_species
    Y = np.full((k, ns), 1e-12)
    w_in = rng.uniform(0.55, 0.75, size=k)
    stab = [mech.oxidiser] + list(mech.products)
    ys = rng.dirichlet(np.full(len(stab), 0.5), size=k)
    rfrac = 10.0 ** rng.uniform(-4.0, -2.0, size=k)
    yr = rng.dirichlet(np.full(len(mech.radicals), 0.5), size=k) if mech.radicals else None
    Y[:, mech.inert] = w_in
    Y[:, stab] += ys * ((1 - w_in) * (1 - rfrac))[:, None]
    if yr is not None:
        Y[:, mech.radicals] += yr * ((1 - w_in) * rfrac)[:, None]
    return Y / Y.sum(axis=1, keepdims=True)


def _noisy(rng, Y: np.ndarray, sigma: float) -> np.ndarray:
    Z = Y * np.exp(rng.normal(0.0, sigma, size=Y.shape))
    return Z / Z.sum(axis=1, keepdims=True)


def generate_states(mech: Mechanism, n_cells: int, pressure: float, recipe: str,
                    seed: int) -> np.ndarray:
    """Cell states phi = [T, p, Y_1..Y_Ns] as a C-contiguous float64 array of
    shape (n_cells, 2 + Ns).

    recipes:
      uniform   - T ~ U[900, 2500] K, Y ~ Dirichlet(1) over all species
      bimodal   - 70% unburnt (T ~ N(800, 50^2) K, fuel U[0.05, 0.3], rest
                  0.23:0.77 oxidiser:inert), 30% hot products-rich cells
                  (T ~ N(2200, 150^2) K, 256 templates with 1% log-normal
                  composition noise and +-5 K)
      ambient   - the bimodal recipe with the same seed, then 60% of the
                  cells (drawn from a second stream, independent of the
                  first) replaced by ambient oxidiser-side gas (Spray A's
                  hot ambient before the spray reaches it): oxidiser:inert
                  0.23:0.77 with the 1e-12 floor of the unburnt cells,
                  T = 900 K + U[-0.5, 0.5] K
      heavytail - T log-spaced over [700, 2600] K, composition blended
                  between unburnt and hot templates by (T-700)/1900; 5% of
                  the cells are ignition-front cells with T ~ U[1100, 1600] K
                  and blend weight U[0.05, 0.5]
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = mech.n_species
    phi = np.empty((n_cells, 2 + ns), dtype=np.float64)
    phi[:, 1] = pressure
    if recipe == "uniform":
        phi[:, 0] = rng.uniform(900.0, 2500.0, size=n_cells)
        phi[:, 2:] = rng.dirichlet(np.ones(ns), size=n_cells)
    elif recipe == "bimodal":
        hot = rng.uniform(size=n_cells) < 0.3
        nh = int(hot.sum())
        T = rng.normal(800.0, 50.0, size=n_cells)
        tmpl = _hot_templates(rng, mech, 256)
        pick = rng.integers(0, 256, size=nh)
        T[hot] = rng.normal(2200.0, 150.0, size=256)[pick] + rng.uniform(-5.0, 5.0, size=nh)
        Y = _unburnt(rng, mech, n_cells)
        Y[hot] = _noisy(rng, tmpl[pick], 0.01)
        phi[:, 0] = T
        phi[:, 2:] = Y
    elif recipe == "ambient":
        phi = generate_states(mech, n_cells, pressure, "bimodal", seed)
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1])))
        amb = rng.uniform(size=n_cells) < 0.6
        na = int(amb.sum())
        Y = np.full(ns, 1e-12)
        Y[mech.oxidiser] = 0.23
        Y[mech.inert] = 0.77
        phi[amb, 0] = 900.0 + rng.uniform(-0.5, 0.5, size=na)
        phi[amb, 2:] = Y / Y.sum()
    elif recipe == "heavytail":
        T = np.exp(np.linspace(math.log(700.0), math.log(2600.0), n_cells))
        rng.shuffle(T)
        w = (T - 700.0) / 1900.0
        front = rng.uniform(size=n_cells) < 0.05
        nf = int(front.sum())
        T[front] = rng.uniform(1100.0, 1600.0, size=nf)
        w[front] = rng.uniform(0.05, 0.5, size=nf)
        tmpl = _hot_templates(rng, mech, 256)
        pick = rng.integers(0, 256, size=n_cells)
        Yu = _unburnt(rng, mech, n_cells)
        Y = (1.0 - w)[:, None] * Yu + w[:, None] * tmpl[pick]
        phi[:, 0] = T
        phi[:, 2:] = Y / Y.sum(axis=1, keepdims=True)
    else:
        raise ValueError("unknown recipe %r" % recipe)
    return np.ascontiguousarray(phi)


def workload_inputs(name: str, directory: str, n_cells: Optional[int] = None):
    """(Workload, Mechanism, mech path, phi) for a named workload. ``n_cells``
    overrides the cell count with a prefix of the same seeded stream."""
    wl = WORKLOADS[name]
    mech, path = mech_cached(wl.mech, directory)
    n = wl.n_cells if n_cells is None else n_cells
    phi = generate_states(mech, wl.n_cells, wl.pressure, wl.recipe, wl.state_seed)
    return wl, mech, path, np.ascontiguousarray(phi[:n])


def sample_indices(n_total: int, n_sample: int, seed: int) -> np.ndarray:
    """Seeded uniform sample (without replacement, sorted) of cell indices."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n_total, size=min(n_sample, n_total), replace=False))
