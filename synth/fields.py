"""Seeded per-cell fields shaped like the paper's hydrogen cases.

All fields are returned as float64 structure-of-arrays: ``T[n]`` (K),
``p[n]`` (Pa) and ``Y[K, n]`` (mass fractions, species-major so that
``Y[k, i]`` is cell i of species k, the layout the library takes with
``ld = n``).

* ``premixed_h2_air(phi)``: H2/air with air O2:N2 = 1:3.76 by moles and
  phi = (n_H2 / n_O2) / 2; radicals and products zero.
* ``ignition_cells`` (1024-cell parity case): T0 ~ U(1000, 1600) K,
  phi ~ U(0.5, 2), p = 1 atm.
* ``hot_kernel_field_2d`` (256 x 256 = 65,536 cells): premixed phi = 1 at
  300 K plus eight Gaussian hot kernels of amplitude U(900, 1500) K and width
  U(4, 16) cells at uniform random centres, capped at 1800 K; p = 1 atm.
  It stands in for the paper's 2-D hydrogen jet/triple-flame field.
* ``mixing_layer_3d`` (100^3 = 1,000,000 cells): a fuel/air mixing layer with
  uneven stiffness for the scheduling study: mixture fraction
  Z = (1 - tanh((y - y0)/delta))/2 + N(0, 0.02^2) clipped to [0, 1]
  (delta = 10 cells, y0 mid-domain), fuel H2/N2 50/50 by moles, oxidiser air;
  progress c = exp(-((Z - Z_st)/0.1)^2) blends the unburnt mixture with its
  complete-combustion products (H2 + O2/2 -> H2O until the deficient reactant
  is used up); T = 300 + 2200 c + N(0, 50^2) clipped to [300, 2500] K;
  p = 1 atm; per-cell dt log-uniform in [1e-7, 1e-5] s.  It stands in for the
  paper's uneven chemistry load across a flame (its DLB motivation).
* ``premixed_ch4_air(phi)``: CH4/air, air O2:N2:AR = 1:3.72:0.0446 by moles
  (21 % O2, 1 % AR), phi = (n_CH4 / n_O2) * 2.
* ``hydrocarbon_field`` (262,144 cells, the 53-species mechanism): T ~ U(300, 2400) K,
  p ~ U(1, 10) atm; composition the blend (1 - c) unburnt + c products of CH4/air at
  phi ~ U(0.5, 1.5) with progress c ~ U(0, 1) (products: CH4 + 2 O2 -> CO2 + 2 H2O until
  the deficient reactant is used up), plus every other species at a mass fraction
  log-uniform in [1e-12, 1e-3], renormalised; dt = 1e-6 s.
"""
from __future__ import annotations

import os

import numpy as np

P_ATM = 101325.0

FIELD_SEED_1 = 1001
FIELD_SEED_2 = 2002
FIELD_SEED_3 = 3003


def premixed_h2_air(mech, phi):
    """Mass fractions [K, n] of H2/air at equivalence ratio phi (array or scalar)."""
    phi = np.atleast_1d(np.asarray(phi, dtype=np.float64))
    K = mech.n_species
    W = np.asarray(mech.molar_mass, dtype=np.float64)
    iH2, iO2, iN2 = mech.index("H2"), mech.index("O2"), mech.index("N2")
    n = np.zeros((K, phi.size))
    n[iH2] = 2.0 * phi
    n[iO2] = 1.0
    n[iN2] = 3.76
    m = n * W[:, None]
    return m / m.sum(axis=0, keepdims=True)


def ignition_cells(mech, n=1024, seed=FIELD_SEED_1, T_range=(1000.0, 1600.0), phi_range=(0.5, 2.0),
                   p=P_ATM):
    rng = np.random.default_rng(seed)
    T = rng.uniform(*T_range, size=n)
    phi = rng.uniform(*phi_range, size=n)
    Y = premixed_h2_air(mech, phi)
    return {"T": T, "p": np.full(n, float(p)), "Y": np.ascontiguousarray(Y), "phi": phi}


def hot_kernel_field_2d(mech, nx=256, ny=256, seed=FIELD_SEED_2, n_kernels=8, T_bg=300.0,
                        amp=(900.0, 1500.0), sigma=(4.0, 16.0), T_cap=1800.0, p=P_ATM):
    rng = np.random.default_rng(seed)
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    T = np.full((ny, nx), T_bg)
    for _ in range(n_kernels):
        a = rng.uniform(*amp)
        s = rng.uniform(*sigma)
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        T = T + a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * s * s))
    T = np.minimum(T, T_cap).reshape(-1)
    n = T.size
    Y = np.repeat(premixed_h2_air(mech, 1.0), n, axis=1)
    return {"T": T, "p": np.full(n, float(p)), "Y": np.ascontiguousarray(Y), "shape": (ny, nx)}


def _mole_to_mass(mech, moles):
    W = np.asarray(mech.molar_mass, dtype=np.float64)
    m = moles * W
    return m / m.sum()


def mixing_layer_3d(mech, n_side=100, seed=FIELD_SEED_3, delta=10.0, z_noise=0.02, T_noise=50.0,
                    dt_range=(1e-7, 1e-5), p=P_ATM):
    rng = np.random.default_rng(seed)
    K = mech.n_species
    iH2, iO2, iH2O, iN2 = mech.index("H2"), mech.index("O2"), mech.index("H2O"), mech.index("N2")
    W = np.asarray(mech.molar_mass, dtype=np.float64)
    xf = np.zeros(K)
    xf[iH2], xf[iN2] = 0.5, 0.5
    xo = np.zeros(K)
    xo[iO2], xo[iN2] = 1.0, 3.76
    Yf, Yo = _mole_to_mass(mech, xf), _mole_to_mass(mech, xo)
    s_ox = 0.5 * W[iO2] / W[iH2]  # kg O2 per kg H2 at stoichiometry
    z_st = Yo[iO2] / (s_ox * Yf[iH2] + Yo[iO2])
    n = n_side ** 3
    yidx = (np.arange(n) // n_side) % n_side  # cell index along y of a (z, y, x) grid
    y0 = 0.5 * (n_side - 1)
    Z = 0.5 * (1.0 - np.tanh((yidx - y0) / delta)) + rng.normal(0.0, z_noise, size=n)
    Z = np.clip(Z, 0.0, 1.0)
    Yu = Z[None, :] * Yf[:, None] + (1.0 - Z)[None, :] * Yo[:, None]
    h2, o2 = Yu[iH2], Yu[iO2]
    burn_h2 = np.minimum(h2, o2 / s_ox)  # H2 burnt, kg per kg of mixture
    Yb = Yu.copy()
    Yb[iH2] = h2 - burn_h2
    Yb[iO2] = o2 - s_ox * burn_h2
    Yb[iH2O] = Yu[iH2O] + (1.0 + s_ox) * burn_h2
    c = np.exp(-((Z - z_st) / 0.1) ** 2)
    Y = (1.0 - c)[None, :] * Yu + c[None, :] * Yb
    Y = np.maximum(Y, 0.0)
    Y /= Y.sum(axis=0, keepdims=True)
    T = np.clip(300.0 + 2200.0 * c + rng.normal(0.0, T_noise, size=n), 300.0, 2500.0)
    dt = np.exp(rng.uniform(np.log(dt_range[0]), np.log(dt_range[1]), size=n))
    return {"T": T, "p": np.full(n, float(p)), "Y": np.ascontiguousarray(Y), "dt": dt, "Z": Z, "c": c,
            "z_st": z_st, "shape": (n_side, n_side, n_side)}


FIELD_SEED_5 = 5005


def premixed_ch4_air(mech, phi):
    """Mass fractions [K, n] of CH4/air at equivalence ratio phi (array or scalar)."""
    phi = np.atleast_1d(np.asarray(phi, dtype=np.float64))
    W = np.asarray(mech.molar_mass, dtype=np.float64)
    n = np.zeros((mech.n_species, phi.size))
    n[mech.index("CH4")] = 0.5 * phi
    n[mech.index("O2")] = 1.0
    n[mech.index("N2")] = 3.72
    n[mech.index("AR")] = 0.0446
    m = n * W[:, None]
    return m / m.sum(axis=0, keepdims=True)


def hydrocarbon_field(mech, n=262144, seed=FIELD_SEED_5, T_range=(300.0, 2400.0), p_range=(1.0, 10.0),
                      phi_range=(0.5, 1.5), minor=(1e-12, 1e-3)):
    rng = np.random.default_rng(seed)
    K = mech.n_species
    W = np.asarray(mech.molar_mass, dtype=np.float64)
    T = rng.uniform(*T_range, size=n)
    p = rng.uniform(*p_range, size=n) * P_ATM
    phi = rng.uniform(*phi_range, size=n)
    c = rng.uniform(0.0, 1.0, size=n)
    iF, iO, iC, iW = mech.index("CH4"), mech.index("O2"), mech.index("CO2"), mech.index("H2O")
    Yu = premixed_ch4_air(mech, phi)
    # complete combustion of the unburnt mixture, per unit mass
    nu = Yu / W[:, None]
    burn = np.minimum(nu[iF], nu[iO] / 2.0)
    nb = nu.copy()
    nb[iF] -= burn
    nb[iO] -= 2.0 * burn
    nb[iC] += burn
    nb[iW] += 2.0 * burn
    Yb = nb * W[:, None]
    Y = (1.0 - c) * Yu + c * Yb
    major = np.zeros(K, dtype=bool)
    major[[iF, iO, iC, iW, mech.index("N2"), mech.index("AR")]] = True
    lo, hi = np.log(minor[0]), np.log(minor[1])
    Y[~major] = np.exp(rng.uniform(lo, hi, size=(int((~major).sum()), n)))
    Y /= Y.sum(axis=0, keepdims=True)
    return {"T": T, "p": p, "Y": np.ascontiguousarray(Y), "phi": phi, "c": c}



SNAPSHOT_S = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "h2_field_snapshot_s.npz")


def snapshot_s(path=SNAPSHOT_S):
    """Snapshot S of the 256 x 256 hot-kernel field: the stored state of the field after the oracle
    integrator advanced it until its hottest cell rose by 500 K (written by
    oracle/make_snapshot_s.py; this only reads it).  Keys as hot_kernel_field_2d, plus h (each
    cell's sub-step hint after the last advancing call) and steps/dt of the advance."""
    z = np.load(path)
    return {"T": z["T"].copy(), "p": z["p"].copy(), "Y": np.ascontiguousarray(z["Y"]), "h": z["h"].copy(),
            "shape": tuple(int(v) for v in z["shape"]), "steps": int(z["steps"]), "dt": float(z["dt"])}
