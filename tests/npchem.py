"""Independent NumPy right-hand side of the constant-pressure reactor (tests only).

Written from the textbook definitions (NASA-7 thermo, mass action with
Arrhenius, third-body and Troe rate constants, equilibrium constants from
Gibbs energies), not from either implementation.  Every operation accepts
complex arguments so that complex-step derivatives can be taken through it.
It is used to pin the oracle's Jacobian (complex step), as the right-hand
side of SciPy's Radau solver, and by the equilibrium and brute-force tests.
"""
from __future__ import annotations

import numpy as np

R = 8.31446261815324
P0 = 101325.0


class NpChem:
    def __init__(self, mech):
        self.m = mech
        self.K = mech.n_species
        self.W = np.asarray(mech.molar_mass, dtype=float) * 1e-3   # kg/mol
        self.a = np.asarray(mech.nasa7, dtype=float)
        self.nu = (mech.nu_prod - mech.nu_reac).astype(float)        # [M, K]

    # -- thermo (molar, dimensionless)
    def cp_R(self, T):
        a = self.a
        return a[:, 0] + a[:, 1] * T + a[:, 2] * T ** 2 + a[:, 3] * T ** 3 + a[:, 4] * T ** 4

    def h_RT(self, T):
        a = self.a
        return (a[:, 0] + a[:, 1] * T / 2 + a[:, 2] * T ** 2 / 3 + a[:, 3] * T ** 3 / 4 + a[:, 4] * T ** 4 / 5
                + a[:, 5] / T)

    def s_R(self, T):
        a = self.a
        return (a[:, 0] * np.log(T) + a[:, 1] * T + a[:, 2] * T ** 2 / 2 + a[:, 3] * T ** 3 / 3
                + a[:, 4] * T ** 4 / 4 + a[:, 6])

    def h_mass(self, T, Y):
        return np.sum(Y * self.h_RT(T) * R * T / self.W)

    def cp_mass(self, T, Y):
        return np.sum(Y * self.cp_R(T) * R / self.W)

    # -- kinetics, concentrations in mol/cm^3
    def kf(self, T, conc):
        m = self.m
        out = []
        for j in range(m.n_reactions):
            A, b, Ta = m.arrhenius[j]
            k = A * T ** b * np.exp(-Ta / T)
            if m.reaction_type[j] == 2:
                M = np.sum(m.efficiency[j] * conc)
                A0, b0, Ta0 = m.falloff_low[j]
                k0 = A0 * T ** b0 * np.exp(-Ta0 / T)
                Pr = k0 * M / k
                al, T3, T1, T2 = m.troe[j]
                Fc = (1 - al) * np.exp(-T / T3) + al * np.exp(-T / T1) + np.exp(-T2 / T)
                c = -0.4 - 0.67 * np.log10(Fc)
                n = 0.75 - 1.27 * np.log10(Fc)
                f1 = (np.log10(Pr) + c) / (n - 0.14 * (np.log10(Pr) + c))
                F = 10.0 ** (np.log10(Fc) / (1 + f1 * f1))
                k = k * Pr / (1 + Pr) * F
            out.append(k)
        return out

    def Kc(self, T):
        g = self.h_RT(T) - self.s_R(T)
        dG = self.nu @ g if not np.iscomplexobj(g) else np.array([np.sum(self.nu[j] * g) for j in range(len(self.nu))])
        dn = self.nu.sum(axis=1)
        return np.exp(-dG) * (P0 / (R * T) * 1e-6) ** dn

    def wdot(self, T, p, Y):
        """Molar production rates, mol/m^3/s."""
        m = self.m
        Wbar = 1.0 / np.sum(Y / self.W)
        rho = p * Wbar / (R * T)
        conc = rho * Y / self.W * 1e-6
        kf = self.kf(T, conc)
        Kc = self.Kc(T)
        w = np.zeros(self.K, dtype=np.result_type(T, Y, complex if np.iscomplexobj(Y) or np.iscomplexobj(T) else float))
        for j in range(m.n_reactions):
            fwd = kf[j] * np.prod(conc ** m.nu_reac[j])
            rev = kf[j] / Kc[j] * np.prod(conc ** m.nu_prod[j])
            q = fwd - rev
            if m.reaction_type[j] == 1:
                q = q * np.sum(m.efficiency[j] * conc)
            w = w + self.nu[j] * q * 1e6
        return w, rho

    def rhs(self, p, y):
        T = y[0]
        Y = y[1:]
        w, rho = self.wdot(T, p, Y)
        dY = self.W * w / rho
        dT = -np.sum(self.h_RT(T) * R * T * w) / (rho * self.cp_mass(T, Y))
        return np.concatenate([[dT], dY])

    def rhs_v(self, rho, y):
        """Constant-volume reactor: rho fixed, p = rho R T / Wbar; the energy equation keeps
        u = sum_k Y_k (H_k - R T)/W_k constant."""
        T = y[0]
        Y = y[1:]
        p = rho * R * T * np.sum(Y / self.W)
        w, _ = self.wdot(T, p, Y)
        dY = self.W * w / rho
        cv = np.sum(Y * (self.cp_R(T) - 1.0) * R / self.W)
        dT = -np.sum((self.h_RT(T) - 1.0) * R * T * w) / (rho * cv)
        return np.concatenate([[dT], dY])

    def u_mass(self, T, Y):
        return np.sum(Y * (self.h_RT(T) - 1.0) * R * T / self.W)

    def jac_v_complex_step(self, rho, y, h=1e-30):
        N = len(y)
        J = np.zeros((N, N))
        for l in range(N):
            yc = np.array(y, dtype=complex)
            step = h * max(abs(y[l]), 1e-3 if l else 1.0)
            yc[l] += 1j * step
            J[:, l] = np.imag(self.rhs_v(rho, yc)) / step
        return J

    def jac_complex_step(self, p, y, h=1e-30):
        N = len(y)
        J = np.zeros((N, N))
        for l in range(N):
            yc = np.array(y, dtype=complex)
            step = h * max(abs(y[l]), 1e-3 if l else 1.0)
            yc[l] += 1j * step
            J[:, l] = np.imag(self.rhs(p, yc)) / step
        return J
