"""Seeded synthetic H2/air-shaped mechanism (9 species, 3 elements, 24 reactions).

The paper's hydrogen mechanisms are not available, so a mechanism of the same
shape is drawn from a seed.  The recipe:

* species H2 O2 H2O H O OH HO2 H2O2 N2, elements H O N with real atomic
  masses; N2 is inert (it only acts as a collision partner);
* the catalogue of element-balanced reversible reactions over the eight
  reactive species with at most two molecules per side and disjoint sides has
  30 entries: 19 two-to-two exchanges and 11 dissociation/recombination
  reactions.  18 of the exchanges and 6 of the recombinations are drawn; 4 of
  those 6 carry a third body (+M) and 2 are Troe falloff reactions (+M).
  Every reaction is written in its exothermic direction (recombinations as
  two -> one), so the drawn rate parameters are those of the exothermic
  direction and the reverse rate from the equilibrium constant is the slower
  one; with random parameters on an endothermic direction the reverse
  constants reach 1e50 and beyond at room temperature;
* Arrhenius parameters: A log-uniform in [1e6, 1e16] (cm-mol-s units),
  b uniform in [-2, 2], Ta = Ea/R uniform in [0, 25000] K;
* third-body efficiencies default to 1, with eps(H2O) in [5, 12] and
  eps(H2) in [1.5, 3];
* Troe: alpha in [0.3, 0.8], T*** in [50, 500] K, T* in [1000, 5000] K,
  T** in [3000, 10000] K; the low-pressure limit k_0 = A0 T^b0 exp(-Ta0/T)
  with b0 in [-2, 0], Ta0 in [0, 5000] K and A0 set so that the reduced
  pressure k_0 [M] / k_inf is log-uniform in [0.1, 10] at 1200 K and 1 atm;
* thermo: one NASA-7 range per species valid over 200-3500 K.  The heat
  capacity template depends on the atom count (1 atom: 2.5; 2 atoms: 3.5 to
  4.5; 3 atoms: 4.0 to 6.5; 4 atoms: 5.0 to 8.0, in units of R, rising
  smoothly from 300 K to 3000 K), perturbed by +-5 % and least-squares fitted
  by a quartic.  a6 and a7 then place the formation enthalpy and the standard
  entropy at 298.15 K in textbook-sized ranges.

Whether a seed gives a mechanism that ignites and equilibrates sensibly is
checked separately (the check needs an integrator); the accepted seed is the
default below.
"""
from __future__ import annotations

import itertools
import numpy as np

from .mechfile import Mechanism

H2_SPECIES = ["H2", "O2", "H2O", "H", "O", "OH", "HO2", "H2O2", "N2"]
H2_ELEMENTS = ["H", "O", "N"]
ATOMIC_MASS = {"H": 1.008, "O": 15.999, "N": 14.007}
H2_COMPOSITION = {
    "H2": (2, 0, 0), "O2": (0, 2, 0), "H2O": (2, 1, 0), "H": (1, 0, 0), "O": (0, 1, 0),
    "OH": (1, 1, 0), "HO2": (1, 2, 0), "H2O2": (2, 2, 0), "N2": (0, 0, 2),
}
# formation enthalpy ranges at 298.15 K, J/mol (textbook magnitudes)
H2_HF_RANGE = {
    "H2": (0.0, 0.0), "O2": (0.0, 0.0), "N2": (0.0, 0.0),
    "H": (200e3, 230e3), "O": (235e3, 260e3), "OH": (30e3, 45e3), "HO2": (5e3, 20e3),
    "H2O": (-250e3, -235e3), "H2O2": (-145e3, -130e3),
}
# standard entropy S(298.15)/R ranges by atom count
S298_RANGE = {1: (13.0, 20.0), 2: (15.0, 25.0), 3: (22.0, 28.0), 4: (26.0, 30.0)}
CP_TEMPLATE = {1: (2.5, 2.5), 2: (3.5, 4.5), 3: (4.0, 6.5), 4: (5.0, 8.0)}

R_GAS = 8.31446261815324          # J/mol/K
P_ATM = 101325.0                  # Pa
T_FIT = (200.0, 3500.0)

DEFAULT_H2_SEED = 20221016        # accepted by oracle/select_mech_seed.py from base 20221014


def reaction_catalogue(species, composition, reactive):
    """Element-balanced reversible reactions with <=2 molecules per side.

    Returns (exchanges, recombinations), each a list of (reactants, products)
    tuples of species indices; recombinations are oriented two -> one.
    """
    idx = [species.index(s) for s in reactive]
    comp = np.asarray(composition)
    sides = [(a,) for a in idx] + [tuple(sorted(c)) for c in itertools.combinations_with_replacement(idx, 2)]

    def elem(side):
        return tuple(comp[list(side)].sum(axis=0))

    found = set()
    for L in sides:
        for R in sides:
            if len(L) == 1 and len(R) == 1:
                continue
            if set(L) & set(R):
                continue
            if elem(L) != elem(R):
                continue
            found.add(tuple(sorted([L, R])))
    exch, recomb = [], []
    for a, b in sorted(found):
        if len(a) == 2 and len(b) == 2:
            exch.append((a, b))
        else:
            two, one = (a, b) if len(a) == 2 else (b, a)
            recomb.append((two, one))
    return exch, recomb


def _cp_template(T, n_atoms, lo_hi, rng):
    lo, hi = lo_hi
    # smooth rise from 300 K to 3000 K
    s = 0.5 * (1.0 + np.tanh((T - 1200.0) / 600.0))
    s0 = 0.5 * (1.0 + np.tanh((300.0 - 1200.0) / 600.0))
    s1 = 0.5 * (1.0 + np.tanh((3000.0 - 1200.0) / 600.0))
    s = (s - s0) / (s1 - s0)
    base = lo + (hi - lo) * s
    if n_atoms == 1:
        base = np.full_like(T, lo)
    scale = 1.0 + rng.uniform(-0.05, 0.05)
    tilt = rng.uniform(-0.05, 0.05) * (T - 1850.0) / 1650.0 * (hi - lo + 0.5)
    return base * scale + tilt


def _fit_nasa7(T, cp_r, hf, s298_r):
    """Least-squares quartic for cp/R, then a6, a7 from H(298.15) and S(298.15)."""
    tau = T / 1000.0                       # fit in T/1000 for a well-conditioned basis
    A = np.vstack([tau ** i for i in range(5)]).T
    c15, *_ = np.linalg.lstsq(A, cp_r, rcond=None)
    a15 = c15 / 1000.0 ** np.arange(5)
    t = 298.15
    h_poly = sum(a15[i] * t ** (i + 1) / (i + 1) for i in range(5))        # H/R without a6
    s_poly = a15[0] * np.log(t) + sum(a15[i] * t ** i / i for i in range(1, 5))
    a6 = hf / R_GAS - h_poly
    a7 = s298_r - s_poly
    return np.concatenate([a15, [a6, a7]])


def generate_h2_mechanism(seed: int = DEFAULT_H2_SEED, n_exchange: int = 18,
                          n_third_body: int = 4, n_troe: int = 2) -> Mechanism:
    rng = np.random.default_rng(seed)
    species = list(H2_SPECIES)
    K = len(species)
    comp = np.array([H2_COMPOSITION[s] for s in species], dtype=int)
    emass = np.array([ATOMIC_MASS[e] for e in H2_ELEMENTS])
    W = comp @ emass

    # ---- thermo
    Tg = np.linspace(*T_FIT, 400)
    nasa = np.zeros((K, 7))
    for k, s in enumerate(species):
        na = int(comp[k].sum())
        cp = _cp_template(Tg, na, CP_TEMPLATE[na], rng)
        hf = rng.uniform(*H2_HF_RANGE[s])
        s298 = rng.uniform(*S298_RANGE[na])
        nasa[k] = _fit_nasa7(Tg, cp, hf, s298)
        cpfit = sum(nasa[k, i] * Tg ** i for i in range(5))
        assert np.all(cpfit > 0.5), f"non-positive cp for {s}"

    # ---- reactions
    exch, recomb = reaction_catalogue(species, comp, species[:8])
    pick_ex = np.sort(rng.choice(len(exch), size=n_exchange, replace=False))
    pick_rc = rng.choice(len(recomb), size=n_third_body + n_troe, replace=False)
    tb_set = np.sort(pick_rc[:n_third_body])
    troe_set = np.sort(pick_rc[n_third_body:])
    rx = [(exch[i], 0) for i in pick_ex] + [(recomb[i], 1) for i in tb_set] + [(recomb[i], 2) for i in troe_set]
    # orient every reaction in its exothermic direction (reaction enthalpy at
    # 298.15 K < 0), so that the drawn Arrhenius parameters never describe the
    # endothermic direction and k_r = k_f / K_c stays below k_f
    h298 = np.array([sum(nasa[k, i] * 298.15 ** (i + 1) / (i + 1) for i in range(5)) + nasa[k, 5]
                     for k in range(K)])
    oriented = []
    for (reac, prod), t in rx:
        dh = sum(h298[s] for s in prod) - sum(h298[s] for s in reac)
        oriented.append(((reac, prod) if dh <= 0 or t != 0 else (prod, reac), t))
    rx = oriented
    M = len(rx)
    rtype = np.zeros(M, dtype=int)
    nu_r = np.zeros((M, K), dtype=int)
    nu_p = np.zeros((M, K), dtype=int)
    arr = np.zeros((M, 3))
    eff = np.ones((M, K))
    low = np.zeros((M, 3))
    troe = np.zeros((M, 4))
    iH2O, iH2 = species.index("H2O"), species.index("H2")
    T_ref = 1200.0
    Cm_ref = P_ATM / (R_GAS * T_ref) * 1e-6      # mol/cm^3 at 1 atm, 1200 K
    for j, ((reac, prod), t) in enumerate(rx):
        rtype[j] = t
        for s in reac:
            nu_r[j, s] += 1
        for s in prod:
            nu_p[j, s] += 1
        arr[j] = (10.0 ** rng.uniform(6.0, 16.0), rng.uniform(-2.0, 2.0), rng.uniform(0.0, 25000.0))
        if t >= 1:
            eff[j, iH2O] = rng.uniform(5.0, 12.0)
            eff[j, iH2] = rng.uniform(1.5, 3.0)
        if t == 2:
            troe[j] = (rng.uniform(0.3, 0.8), rng.uniform(50.0, 500.0),
                       rng.uniform(1000.0, 5000.0), rng.uniform(3000.0, 10000.0))
            b0 = rng.uniform(-2.0, 0.0)
            ta0 = rng.uniform(0.0, 5000.0)
            pr = 10.0 ** rng.uniform(-1.0, 1.0)
            A, b, Ta = arr[j]
            kinf = A * T_ref ** b * np.exp(-Ta / T_ref)
            A0 = pr * kinf / (Cm_ref * T_ref ** b0 * np.exp(-ta0 / T_ref))
            low[j] = (A0, b0, ta0)
    # element balance is a property of the catalogue; assert it anyway
    assert np.all((nu_p - nu_r) @ comp == 0)
    return Mechanism(name="h2_synth_9sp_24r", seed=int(seed), elements=list(H2_ELEMENTS),
                     element_mass=emass, species=species, molar_mass=W, composition=comp,
                     nasa7=nasa, reaction_type=rtype, nu_reac=nu_r, nu_prod=nu_p, arrhenius=arr,
                     efficiency=eff, falloff_low=low, troe=troe)
