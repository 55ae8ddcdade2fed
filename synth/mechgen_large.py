"""Seeded synthetic hydrocarbon-shaped mechanism (53 species, 5 elements, 325 reactions).

The paper expects the DNN's advantage to grow with complex hydrocarbon mechanisms;
none is available here, so one of that shape is drawn from a seed.  The recipe:

* elements C H O N Ar with real atomic masses;
* species: a fixed core of 13 (H2 O2 H2O H O OH HO2 H2O2 N2 AR CH4 CO CO2) plus 40
  compositions C_c H_h O_o N_n drawn without replacement from every composition with
  c <= 3, o <= 2, n <= 2, 2 to 10 atoms, h <= 2c + n + 2 (no more hydrogen than a
  saturated skeleton holds) and at least one C or N, weighted 3:1 towards carbon; each
  species is named by its formula.  Only AR is inert;
* reactions: the catalogue of element-balanced reversible reactions over the 52 reactive
  species with at most two molecules per side and disjoint sides; 270 two-to-two
  exchanges, 25 third-body recombinations (+M) and 30 Troe falloff recombinations
  are drawn, and a draw is repeated until every reactive species takes part in some
  reaction.  Exchanges are written in the direction of negative Gibbs energy of reaction
  at 1000 K; third-body and falloff reactions (one molecule <-> two) in the direction of
  negative reaction enthalpy at 298.15 K (a recombination where forming the bond releases
  heat, else a dissociation).  Either way
  the drawn rate parameters describe the favoured direction and the reverse rate from
  the equilibrium constant is the slower one (a recombination of two closed-shell
  molecules into a less stable one, written as a recombination, would have a dissociation
  rate of 1e26 /s);
* Arrhenius parameters as for the hydrogen mechanism but with A log-uniform in
  [1e6, 1e14] (cm-mol-s units; about the collision limit), third-body efficiencies (eps(H2O) in [5, 12], eps(H2) in
  [1.5, 3], eps(CO2) in [2, 4], eps(CH4) in [1.5, 3], eps(AR) in [0.5, 1]) and Troe
  parameters as for the hydrogen mechanism;
* thermo: one NASA-7 range per species over 200-3500 K from the hydrogen mechanism's
  heat-capacity template, extended to n atoms (cp/R from 4.0 + 0.6 (n - 3) at 300 K
  rising to 3 n - 3.5 at 3000 K), least-squares fitted by a quartic; formation
  enthalpies of the core in textbook-sized ranges, of the drawn species from atom
  increments (C +10..40, H -15..-5, O -130..-80, N +20..60 kJ/mol), +100..200 kJ/mol for
  an odd electron count (a radical), and 400..720 kJ/mol for a single atom; S(298)/R by
  atom count.

Whether a seed gives a mechanism that ignites and equilibrates sensibly is checked
separately with the oracle (oracle/select_large_mech_seed.py); the accepted seed is the
default below.
"""
from __future__ import annotations

import itertools

import numpy as np

from .mechfile import Mechanism
from .mechgen import R_GAS, P_ATM, T_FIT, _fit_nasa7

ELEMENTS = ["C", "H", "O", "N", "AR"]
ATOMIC_MASS = {"C": 12.011, "H": 1.008, "O": 15.999, "N": 14.007, "AR": 39.948}
CORE = {
    "H2": (0, 2, 0, 0, 0), "O2": (0, 0, 2, 0, 0), "H2O": (0, 2, 1, 0, 0), "H": (0, 1, 0, 0, 0),
    "O": (0, 0, 1, 0, 0), "OH": (0, 1, 1, 0, 0), "HO2": (0, 1, 2, 0, 0), "H2O2": (0, 2, 2, 0, 0),
    "N2": (0, 0, 0, 2, 0), "AR": (0, 0, 0, 0, 1), "CH4": (1, 4, 0, 0, 0), "CO": (1, 0, 1, 0, 0),
    "CO2": (1, 0, 2, 0, 0),
}
# formation enthalpy ranges at 298.15 K, J/mol (textbook magnitudes)
CORE_HF = {
    "H2": (0.0, 0.0), "O2": (0.0, 0.0), "N2": (0.0, 0.0), "AR": (0.0, 0.0),
    "H": (200e3, 230e3), "O": (235e3, 260e3), "OH": (30e3, 45e3), "HO2": (5e3, 20e3),
    "H2O": (-250e3, -235e3), "H2O2": (-145e3, -130e3), "CH4": (-80e3, -70e3),
    "CO": (-115e3, -105e3), "CO2": (-400e3, -385e3),
}
N_DRAWN = 40
DEFAULT_LARGE_SEED = 20221112        # accepted by oracle/select_large_mech_seed.py from base 20221101


def _formula(c):
    parts = []
    for e, n in zip(("C", "H", "O", "N"), c[:4]):
        if n:
            parts.append(e if n == 1 else f"{e}{n}")
    return "".join(parts)


def candidate_compositions():
    out = []
    for c in range(4):
        for o in range(3):
            for n in range(3):
                for h in range(9):
                    na = c + h + o + n
                    if na < 2 or na > 10 or (c == 0 and n == 0):
                        continue
                    if h > 2 * c + n + 2:
                        continue
                    comp = (c, h, o, n, 0)
                    if comp in CORE.values():
                        continue
                    out.append(comp)
    return out


def _cp_range(na):
    if na <= 4:
        return {1: (2.5, 2.5), 2: (3.5, 4.5), 3: (4.0, 6.5), 4: (5.0, 8.0)}[na]
    return (4.0 + 0.6 * (na - 3), 3.0 * na - 3.5)


def _s298_range(na):
    if na <= 4:
        return {1: (13.0, 20.0), 2: (15.0, 25.0), 3: (22.0, 28.0), 4: (26.0, 30.0)}[na]
    return (26.0 + 3.0 * (na - 4), 30.0 + 3.5 * (na - 4))


def _cp_curve(T, na, rng):
    lo, hi = _cp_range(na)
    s = 0.5 * (1.0 + np.tanh((T - 1200.0) / 600.0))
    s0 = 0.5 * (1.0 + np.tanh((300.0 - 1200.0) / 600.0))
    s1 = 0.5 * (1.0 + np.tanh((3000.0 - 1200.0) / 600.0))
    s = (s - s0) / (s1 - s0)
    base = np.full_like(T, lo) if na == 1 else lo + (hi - lo) * s
    scale = 1.0 + rng.uniform(-0.05, 0.05)
    tilt = rng.uniform(-0.05, 0.05) * (T - 1850.0) / 1650.0 * (hi - lo + 0.5)
    return base * scale + tilt


def _catalogue(comp, reactive):
    sides = [(a,) for a in reactive] + [tuple(c) for c in itertools.combinations_with_replacement(reactive, 2)]
    by_elem = {}
    for s in sides:
        by_elem.setdefault(tuple(comp[list(s)].sum(axis=0)), []).append(s)
    exch, recomb = [], []
    for group in by_elem.values():
        for a, b in itertools.combinations(group, 2):
            if set(a) & set(b) or (len(a) == 1 and len(b) == 1):
                continue
            if len(a) == 2 and len(b) == 2:
                exch.append((a, b))
            else:
                recomb.append((a, b) if len(a) == 2 else (b, a))
    return exch, recomb


def generate_large_mechanism(seed: int = DEFAULT_LARGE_SEED, n_exchange: int = 270, n_third_body: int = 25,
                             n_troe: int = 30) -> Mechanism:
    rng = np.random.default_rng(seed)
    cands = candidate_compositions()
    w = np.array([3.0 if c[0] > 0 else 1.0 for c in cands])
    pick = rng.choice(len(cands), size=N_DRAWN, replace=False, p=w / w.sum())
    drawn = sorted((cands[i] for i in pick), key=lambda c: (c[0], c[3], c[2], c[1]))
    species = list(CORE) + [_formula(c) for c in drawn]
    comp = np.array([CORE[s] for s in CORE] + list(drawn), dtype=int)
    K = len(species)
    emass = np.array([ATOMIC_MASS[e] for e in ELEMENTS])
    W = comp @ emass

    # ---- thermo
    Tg = np.linspace(*T_FIT, 400)
    nasa = np.zeros((K, 7))
    for k, s in enumerate(species):
        c, h, o, n, ar = comp[k]
        na = int(comp[k].sum())
        cp = _cp_curve(Tg, na, rng)
        if s in CORE_HF:
            hf = rng.uniform(*CORE_HF[s])
        elif na == 1:
            hf = rng.uniform(400e3, 720e3)
        else:
            hf = 1e3 * (c * rng.uniform(10, 40) - h * rng.uniform(5, 15) - o * rng.uniform(80, 130)
                        + n * rng.uniform(20, 60))
            if (4 * c + h + 2 * o + 3 * n) % 2 == 1:
                hf += rng.uniform(100e3, 200e3)
        s298 = rng.uniform(*_s298_range(na))
        nasa[k] = _fit_nasa7(Tg, cp, hf, s298)
        cpfit = sum(nasa[k, i] * Tg ** i for i in range(5))
        assert np.all(cpfit > 0.5), f"non-positive cp for {s}"

    # ---- reactions
    iAR = species.index("AR")
    reactive = [k for k in range(K) if k != iAR]
    exch, recomb = _catalogue(comp, reactive)
    h298 = np.array([sum(nasa[k, i] * 298.15 ** (i + 1) / (i + 1) for i in range(5)) + nasa[k, 5]
                     for k in range(K)]) * R_GAS
    T1 = 1000.0
    g1 = np.array([sum(nasa[k, i] * T1 ** i / (i + 1) for i in range(5)) + nasa[k, 5] / T1
                   - (nasa[k, 0] * np.log(T1) + sum(nasa[k, i] * T1 ** i / i for i in range(1, 5)) + nasa[k, 6])
                   for k in range(K)])                                   # G/RT at 1000 K
    recomb = [((two, one) if h298[one[0]] - h298[two[0]] - h298[two[1]] < 0.0 else (one, two)) for two, one in recomb]
    if len(recomb) < n_third_body + n_troe:
        raise ValueError(f"seed {seed}: only {len(recomb)} one <-> two reactions")
    for _ in range(1000):
        pe = np.sort(rng.choice(len(exch), size=n_exchange, replace=False))
        pr = rng.choice(len(recomb), size=n_third_body + n_troe, replace=False)
        used = set()
        for i in pe:
            used.update(exch[i][0] + exch[i][1])
        for i in pr:
            used.update(recomb[i][0] + recomb[i][1])
        if used >= set(reactive):
            break
    else:
        raise RuntimeError("no draw covers every reactive species")
    rx = [(exch[i], 0) for i in pe] + [(recomb[i], 1) for i in np.sort(pr[:n_third_body])] + \
         [(recomb[i], 2) for i in np.sort(pr[n_third_body:])]
    rx = [(((r, p) if t != 0 or sum(g1[s] for s in p) - sum(g1[s] for s in r) <= 0 else (p, r)), t)
          for (r, p), t in rx]
    M = len(rx)
    rtype = np.zeros(M, dtype=int)
    nu_r = np.zeros((M, K), dtype=int)
    nu_p = np.zeros((M, K), dtype=int)
    arr = np.zeros((M, 3))
    eff = np.ones((M, K))
    low = np.zeros((M, 3))
    troe = np.zeros((M, 4))
    idx = {s: species.index(s) for s in ("H2O", "H2", "CO2", "CH4", "AR")}
    T_ref = 1200.0
    Cm_ref = P_ATM / (R_GAS * T_ref) * 1e-6
    for j, ((reac, prod), t) in enumerate(rx):
        rtype[j] = t
        for s in reac:
            nu_r[j, s] += 1
        for s in prod:
            nu_p[j, s] += 1
        arr[j] = (10.0 ** rng.uniform(6.0, 14.0), rng.uniform(-2.0, 2.0), rng.uniform(0.0, 25000.0))
        if t >= 1:
            eff[j, idx["H2O"]] = rng.uniform(5.0, 12.0)
            eff[j, idx["H2"]] = rng.uniform(1.5, 3.0)
            eff[j, idx["CO2"]] = rng.uniform(2.0, 4.0)
            eff[j, idx["CH4"]] = rng.uniform(1.5, 3.0)
            eff[j, idx["AR"]] = rng.uniform(0.5, 1.0)
        if t == 2:
            troe[j] = (rng.uniform(0.3, 0.8), rng.uniform(50.0, 500.0),
                       rng.uniform(1000.0, 5000.0), rng.uniform(3000.0, 10000.0))
            b0 = rng.uniform(-2.0, 0.0)
            ta0 = rng.uniform(0.0, 5000.0)
            prr = 10.0 ** rng.uniform(-1.0, 1.0)
            A, b, Ta = arr[j]
            kinf = A * T_ref ** b * np.exp(-Ta / T_ref)
            low[j] = (prr * kinf / (Cm_ref * T_ref ** b0 * np.exp(-ta0 / T_ref)), b0, ta0)
    assert np.all((nu_p - nu_r) @ comp == 0)
    return Mechanism(name="hc_synth_53sp_325r", seed=int(seed), elements=list(ELEMENTS), element_mass=emass,
                     species=species, molar_mass=W, composition=comp, nasa7=nasa, reaction_type=rtype,
                     nu_reac=nu_r, nu_prod=nu_p, arrhenius=arr, efficiency=eff, falloff_low=low, troe=troe)
