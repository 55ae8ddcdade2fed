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
"""
from __future__ import annotations

import numpy as np

P_ATM = 101325.0

FIELD_SEED_1 = 1001
FIELD_SEED_2 = 2002


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
