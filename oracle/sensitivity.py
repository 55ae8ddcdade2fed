"""Forward sensitivities of one chemistry step -- test infrastructure only.

The discrete adjoint of the step is checked against the derivatives computed
here: d y(dt) / d(T0, Y0, ln A_j) of the RODAS4 integration of the
constant-pressure reactor with its accepted sub-step lengths held fixed (the
step-size controller's choices are part of the sequence, not differentiated;
a replay of the sequence with every input nudged is a smooth function of the
inputs).

Method, in the order the derivative is built:
  * the right-hand side f(y; ln A) of the reactor (species source term of the
    paper's Sec. "Chemistry Integration", the energy equation at constant
    enthalpy, NASA-7 thermo, Arrhenius / third-body / Troe rate constants and
    equilibrium constants from Gibbs energies) is written once, vectorised
    over reactions and over a batch of states, with operations that accept
    complex numbers and forward-mode dual numbers alike;
  * the Jacobian J = df/dy inside each sub-step is the exact derivative of
    that f, taken by forward-mode automatic differentiation (dual numbers
    with one direction per state component), so it is available at complex
    states too;
  * each input direction is a separate replay of the sub-steps in complex
    arithmetic with that input nudged by i*h, h = 1e-30; the derivative is
    Im(y(dt)) / h, exact to rounding because no difference of nearby values
    is formed (complex-step differentiation: Squire and Trapp, SIAM Review
    40 (1998); Martins, Sturdza and Alonso, ACM TOMS 29 (2003)).
The 1 + K inputs (T0, Y0) and the M log pre-exponential factors (for Troe
rows the high-pressure limit k_inf) run together as one batch of complex
replays.  The RODAS4 coefficients are the oracle's own table.

Shares nothing with the GPU library; plain NumPy, slow and direct.
"""
from __future__ import annotations

import numpy as np

R = 8.31446261815324   # J/mol/K
P0 = 101325.0          # Pa, standard state of the NASA-7 fits
LN10 = np.log(10.0)
H_CS = 1e-30


class Dual:
    """Forward-mode dual number: value a and derivatives b, b.shape == a.shape + (D,)."""

    __array_ufunc__ = None  # make NumPy defer to the reflected operators below

    def __init__(self, a, b):
        self.a = a
        self.b = b

    # -- helpers
    @staticmethod
    def _split(x):
        if isinstance(x, Dual):
            return x.a, x.b
        return x, None

    def __getitem__(self, idx):
        if not isinstance(idx, tuple):
            idx = (idx,)
        return Dual(self.a[idx], self.b[idx + (slice(None),)])

    def __neg__(self):
        return Dual(-self.a, -self.b)

    def __add__(self, o):
        oa, ob = self._split(o)
        a = self.a + oa
        b = self.b + ob if ob is not None else self.b + np.zeros(np.shape(oa))[..., None]
        return Dual(a, np.broadcast_to(b, a.shape + self.b.shape[-1:]))

    __radd__ = __add__

    def __sub__(self, o):
        return self + (-o)

    def __rsub__(self, o):
        return (-self) + o

    def __mul__(self, o):
        oa, ob = self._split(o)
        a = self.a * oa
        if ob is None:
            b = self.b * np.asarray(oa)[..., None]
        else:
            b = self.b * np.asarray(oa)[..., None] + ob * np.asarray(self.a)[..., None]
        return Dual(a, np.broadcast_to(b, np.shape(a) + self.b.shape[-1:]))

    __rmul__ = __mul__

    def reciprocal(self):
        r = 1.0 / self.a
        return Dual(r, -self.b * (r * r)[..., None])

    def __truediv__(self, o):
        if isinstance(o, Dual):
            return self * o.reciprocal()
        return self * (1.0 / np.asarray(o))

    def __rtruediv__(self, o):
        return self.reciprocal() * o

    def sum(self, axis):
        return Dual(self.a.sum(axis=axis), self.b.sum(axis=axis))


def exp(x):
    if isinstance(x, Dual):
        e = np.exp(x.a)
        return Dual(e, x.b * e[..., None])
    return np.exp(x)


def log(x):
    if isinstance(x, Dual):
        return Dual(np.log(x.a), x.b / x.a[..., None])
    return np.log(x)


def where(mask, x, y):
    """Elementwise choice along the last axis of the values (mask broadcasts against them)."""
    if isinstance(x, Dual) or isinstance(y, Dual):
        xa, xb = Dual._split(x)
        ya, yb = Dual._split(y)
        D = (xb if xb is not None else yb).shape[-1]
        shape = np.broadcast_shapes(np.shape(xa), np.shape(ya), np.shape(mask))
        if xb is None:
            xb = np.zeros(shape + (D,))
        if yb is None:
            yb = np.zeros(shape + (D,))
        return Dual(np.where(mask, xa, ya), np.where(np.asarray(mask)[..., None], xb, yb))
    return np.where(mask, x, y)


def concat(parts, axis):
    if any(isinstance(p, Dual) for p in parts):
        return Dual(np.concatenate([p.a for p in parts], axis=axis), np.concatenate([p.b for p in parts], axis=axis))
    return np.concatenate(parts, axis=axis)


def matmul_const(x, Mat):
    """x[..., k] @ Mat[k, m] with a constant matrix."""
    if isinstance(x, Dual):
        return Dual(x.a @ Mat, np.einsum("...kd,km->...md", x.b, Mat))
    return x @ Mat


def ipow(x, n):
    """x[..., None] ** n[m] for small non-negative integer exponents n (by multiplication)."""
    xe = x[:, None]
    out = 1.0
    for e in range(1, int(n.max(initial=0)) + 1):
        out = where(n >= e, xe * out, out) if e > 1 else where(n >= 1, xe, 1.0)
    return out


class Kinetics:
    """The reactor right-hand side of one mechanism (synth.Mechanism), batched over states."""

    def __init__(self, mech):
        self.K = mech.n_species
        self.M = mech.n_reactions
        self.N = self.K + 1
        self.W = np.asarray(mech.molar_mass, dtype=float) * 1e-3
        self.a = np.asarray(mech.nasa7, dtype=float)
        self.nu_r = np.asarray(mech.nu_reac, dtype=int)
        self.nu_p = np.asarray(mech.nu_prod, dtype=int)
        self.nu = (self.nu_p - self.nu_r).astype(float)          # [M, K]
        self.dnu = self.nu.sum(axis=1)
        self.type = np.asarray(mech.reaction_type, dtype=int)
        arr = np.asarray(mech.arrhenius, dtype=float)
        self.lnA, self.b, self.Ta = np.log(arr[:, 0]), arr[:, 1], arr[:, 2]
        self.eff = np.asarray(mech.efficiency, dtype=float)      # [M, K]
        self.troe_rows = np.nonzero(self.type == 2)[0]
        self.other_rows = np.nonzero(self.type != 2)[0]
        lo = np.asarray(mech.falloff_low, dtype=float)[self.troe_rows]
        self.lnA0, self.b0, self.Ta0 = np.log(lo[:, 0]), lo[:, 1], lo[:, 2]
        self.troe = np.asarray(mech.troe, dtype=float)[self.troe_rows]
        # kf of the combined (other, troe) column order back to reaction order
        self.perm = np.argsort(np.concatenate([self.other_rows, self.troe_rows]))

    def rhs(self, x, p, dlnA=None):
        """f(y) for a batch of states x[B, N] (array, complex array or Dual); dlnA[B, M] offsets of ln A."""
        a = self.a
        T = x[:, 0]
        Y = x[:, 1:]
        Tc = T[:, None]
        iT = 1.0 / T
        lnT = log(T)
        # NASA-7 thermo per species, dimensionless
        cpR = a[:, 0] + Tc * (a[:, 1] + Tc * (a[:, 2] + Tc * (a[:, 3] + Tc * a[:, 4])))
        hRT = a[:, 0] + Tc * (a[:, 1] / 2 + Tc * (a[:, 2] / 3 + Tc * (a[:, 3] / 4 + Tc * a[:, 4] / 5))) \
            + a[:, 5] * iT[:, None]
        sR = a[:, 0] * lnT[:, None] + Tc * (a[:, 1] + Tc * (a[:, 2] / 2 + Tc * (a[:, 3] / 3 + Tc * a[:, 4] / 4))) \
            + a[:, 6]
        gRT = hRT - sR
        # mixture
        Wbar = 1.0 / (Y / self.W).sum(axis=1)
        rho = p * Wbar * iT / R
        cp = (Y * cpR * (R / self.W)).sum(axis=1)
        c = 1e-6 * rho[:, None] * Y / self.W                       # mol/cm^3
        # rate constants
        lnk = self.lnA + self.b * lnT[:, None] - self.Ta * iT[:, None]
        if dlnA is not None:
            lnk = lnk + dlnA
        kinf = exp(lnk)
        Mc = matmul_const(c, self.eff.T)                            # third-body concentration [B, M]
        kf = kinf
        if self.troe_rows.size:
            tr = self.troe_rows
            k0 = exp(self.lnA0 + self.b0 * lnT[:, None] - self.Ta0 * iT[:, None])
            Pr = k0 * Mc[:, tr] / kinf[:, tr]
            al, T3, T1, T2 = self.troe.T
            Fc = (1 - al) * exp(-Tc / T3) + al * exp(-Tc / T1) + exp(-T2 * iT[:, None])
            lFc = log(Fc) / LN10
            cc = -0.4 - 0.67 * lFc
            nn = 0.75 - 1.27 * lFc
            xx = log(Pr) / LN10 + cc
            f1 = xx / (nn - 0.14 * xx)
            F = exp(LN10 * lFc / (1.0 + f1 * f1))
            kt = kinf[:, tr] * Pr / (1.0 + Pr) * F
            kf = concat([kinf[:, self.other_rows], kt], axis=1)[:, self.perm]
        # reverse rate constants from the equilibrium constant in concentration units
        lnKc = -matmul_const(gRT, self.nu.T) + self.dnu * log(1e-6 * P0 / R * iT)[:, None]
        kr = kf * exp(-lnKc)
        # mass action, cycling over species (each factor c_k^nu per reaction)
        Pf, Pb = 1.0, 1.0
        for k in range(self.K):
            Pf = ipow(c[:, k], self.nu_r[:, k]) * Pf
            Pb = ipow(c[:, k], self.nu_p[:, k]) * Pb
        q = kf * Pf - kr * Pb
        q = where(self.type == 1, q * Mc, q)
        wdot = 1e6 * matmul_const(q, self.nu)                       # mol/m^3/s
        fY = wdot * self.W / rho[:, None]
        fT = -(hRT * wdot).sum(axis=1) * R * T / (rho * cp)
        return concat([fT[:, None], fY], axis=1)

    def jacobian(self, y, p, dlnA=None):
        """Exact df/dy at a batch of (real or complex) states y[B, N], by forward-mode dual numbers."""
        B, N = y.shape
        eye = np.broadcast_to(np.eye(N), (B, N, N)).astype(y.dtype)
        f = self.rhs(Dual(y, eye), p, dlnA)
        return f.b                                                  # [B, N_out, N_in]


def sensitivities(kin: Kinetics, tableau, p, y0, hs):
    """Replay of the sub-steps hs from y0 = (T0, Y0) with every input nudged in turn.

    Returns (y_end, S) with y_end the replayed state and S[N, N + M] = d y_end / d(T0, Y0, ln A)."""
    gamma, A, Cc, Mw, _ = tableau
    N, M = kin.N, kin.M
    B = N + M
    y = np.tile(np.asarray(y0, dtype=complex), (B, 1))
    y[np.arange(N), np.arange(N)] += 1j * H_CS
    dlnA = np.zeros((B, M), dtype=complex)
    dlnA[N + np.arange(M), np.arange(M)] = 1j * H_CS
    I = np.eye(N)
    for h in hs:
        Wm = I / (gamma * h) - kin.jacobian(y, p, dlnA)
        u = []
        for s in range(6):
            ys = y + sum(A[s, j] * u[j] for j in range(s)) if s else y
            r = kin.rhs(ys, p, dlnA) + sum((Cc[s, j] / h) * u[j] for j in range(s))
            u.append(np.linalg.solve(Wm, r[..., None])[..., 0])
        y = y + sum(Mw[s] * u[s] for s in range(6))
    return y[0].real.copy(), (y.imag / H_CS).T.copy()
