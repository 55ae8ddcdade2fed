"""CPU oracle of the per-cell chemistry step -- test infrastructure only.

Python access (ctypes, numpy arrays) to the plain FP64 C implementation in
``oracle.c``.  Only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use it; the GPU library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# DF_ORACLE_NATIVE=1 selects a build of the same source at -O3 -march=native (the CPU baseline of
# the benchmark, timed on the host it runs on); the default build is plain -O2
NATIVE = os.environ.get("DF_ORACLE_NATIVE", "") == "1"
LIB_PATH = os.path.join(HERE, "liboracle_native.so" if NATIVE else "liboracle.so")
FLAGS = ["-O3", "-march=native"] if NATIVE else ["-O2"]

STATUS = {0: "OK", 1: "MAX_STEPS", 2: "H_UNDERFLOW", 3: "NONFINITE", 4: "DNN_FALLBACK"}


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, or -O3 -march=native with DF_ORACLE_NATIVE=1; OpenMP
    over cells)."""
    cmd = ["gcc", *FLAGS, "-std=c99", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wno-unused-result",
           os.path.join(HERE, "oracle.c"), "-o", LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol_T", C.c_double), ("atol_Y", C.c_double), ("h_min", C.c_double),
                ("max_steps", C.c_int32)]


def default_opts(**kw) -> _Opts:
    o = _Opts(1e-8, 1e-6, 1e-14, 1e-20, 100000)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    # the -march=native build is made on the host that runs it, once per process
    if NATIVE or not os.path.exists(LIB_PATH) or \
            os.path.getmtime(LIB_PATH) < os.path.getmtime(os.path.join(HERE, "oracle.c")):
        build()
    L = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    vp = C.c_void_p
    L.orc_mech_load.restype = vp
    L.orc_mech_load.argtypes = [C.c_char_p]
    L.orc_mech_free.argtypes = [vp]
    L.orc_mech_dims.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.orc_species_thermo.argtypes = [vp, C.c_double, dp, dp, dp, dp]
    L.orc_mixture.argtypes = [vp, C.c_double, C.c_double, dp, dp, dp, dp, dp]
    L.orc_rates.argtypes = [vp, C.c_double, C.c_double, dp, dp, dp, dp, dp]
    L.orc_rhs.argtypes = [vp, C.c_double, dp, dp]
    L.orc_jacobian.argtypes = [vp, C.c_double, dp, dp]
    L.orc_rodas4_tableau.argtypes = [dp, dp, dp, dp, dp]
    L.orc_linear_integrate.restype = C.c_int
    L.orc_linear_integrate.argtypes = [C.c_int, dp, dp, C.c_double, C.c_double, C.POINTER(_Opts), dp, dp, ip, ip]
    L.orc_linear_fixed_step.argtypes = [C.c_int, dp, dp, C.c_double, dp]
    L.orc_chem_step.restype = C.c_int
    L.orc_chem_step.argtypes = [vp, C.c_int64, C.c_int64, C.c_double, dp, dp, dp, dp, dp, ip, ip, ip,
                                C.POINTER(_Opts), C.c_int]
    L.orc_chem_step_dt.restype = C.c_int
    L.orc_chem_step_dt.argtypes = [vp, C.c_int64, C.c_int64, C.c_double, dp, dp, dp, dp, dp, dp, ip, ip, ip,
                                   C.POINTER(_Opts), C.c_int]
    L.orc_rhs_v.argtypes = [vp, C.c_double, dp, dp]
    L.orc_jacobian_v.argtypes = [vp, C.c_double, dp, dp]
    L.orc_chem_step_v.restype = C.c_int
    L.orc_chem_step_v.argtypes = [vp, C.c_int64, C.c_int64, C.c_double, dp, dp, dp, dp, ip, ip, ip,
                                  C.POINTER(_Opts), C.c_int]
    L.orc_chem_cell_record.restype = C.c_int
    L.orc_chem_cell_record.argtypes = [vp, C.c_double, C.c_double, dp, C.POINTER(_Opts), dp, C.c_int32, ip, ip]
    L.orc_chem_replay.argtypes = [vp, C.c_double, dp, dp, C.c_int32]
    L.orc_mech_scale_A.argtypes = [vp, C.c_int32, C.c_double]
    L.orc_dnn_load.restype = vp
    L.orc_dnn_load.argtypes = [C.c_char_p]
    L.orc_dnn_free.argtypes = [vp]
    L.orc_dnn_dims.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), dp, dp]
    L.orc_bct.restype = C.c_double
    L.orc_bct.argtypes = [C.c_double, C.c_double]
    L.orc_bct_inv.restype = C.c_double
    L.orc_bct_inv.argtypes = [C.c_double, C.c_double]
    L.orc_bf16_round.restype = C.c_float
    L.orc_bf16_round.argtypes = [C.c_float]
    L.orc_mlp_forward.argtypes = [vp, dp, dp, C.c_int]
    L.orc_fp8_e4m3_round.restype = C.c_double
    L.orc_fp8_e4m3_round.argtypes = [C.c_double]
    L.orc_fp8_scale_exp.restype = C.c_int
    L.orc_fp8_scale_exp.argtypes = [C.c_double]
    L.orc_mlp_forward_fp8.argtypes = [vp, C.c_int64, dp, dp]
    L.orc_T_from_h.restype = C.c_int
    L.orc_T_from_h.argtypes = [vp, C.c_double, dp, C.c_double, dp]
    L.orc_dnn_step.restype = C.c_int
    L.orc_dnn_step.argtypes = [vp, vp, C.c_int64, C.c_int64, C.c_double, dp, dp, dp, dp, ip, C.c_int, C.c_int,
                               C.c_int, C.POINTER(_Opts), C.c_int]
    _lib = L
    return L


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class Mech:
    """Oracle mechanism handle."""

    def __init__(self, path):
        self.path = str(path)
        self._h = lib().orc_mech_load(self.path.encode())
        if not self._h:
            raise ValueError(f"oracle: cannot load mechanism {path}")
        K, M, E = C.c_int(), C.c_int(), C.c_int()
        lib().orc_mech_dims(self._h, C.byref(K), C.byref(M), C.byref(E))
        self.K, self.M, self.E = K.value, M.value, E.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_mech_free(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def thermo(self, T):
        K = self.K
        cp, h, s, g = (np.zeros(K) for _ in range(4))
        lib().orc_species_thermo(self._h, float(T), _dp(cp), _dp(h), _dp(s), _dp(g))
        return cp, h, s, g

    def mixture(self, T, p, Y):
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        out = [C.c_double() for _ in range(4)]
        lib().orc_mixture(self._h, float(T), float(p), _dp(Y), *[C.byref(o) for o in out])
        return tuple(o.value for o in out)  # Wbar, rho, cp_mass, h_mass

    def rates(self, T, p, Y):
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        kf, kr, q = np.zeros(self.M), np.zeros(self.M), np.zeros(self.M)
        wdot = np.zeros(self.K)
        lib().orc_rates(self._h, float(T), float(p), _dp(Y), _dp(kf), _dp(kr), _dp(q), _dp(wdot))
        return kf, kr, q, wdot

    def rhs(self, p, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        f = np.zeros(self.K + 1)
        lib().orc_rhs(self._h, float(p), _dp(y), _dp(f))
        return f

    def jacobian(self, p, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        N = self.K + 1
        J = np.zeros((N, N))
        lib().orc_jacobian(self._h, float(p), _dp(y), _dp(J))
        return J

    def chem_step(self, T, p, Y, dt, h_inout=None, want_rr=False, opts=None, nthreads=0):
        """Advance all cells by dt (scalar, or one value per cell).  T[n], p[n], Y[K, n] (copied); returns dict."""
        T = np.array(T, dtype=np.float64, copy=True)
        p = np.ascontiguousarray(p, dtype=np.float64)
        Y = np.array(Y, dtype=np.float64, copy=True, order="C")
        n = T.size
        assert Y.shape == (self.K, n)
        h = None if h_inout is None else np.array(h_inout, dtype=np.float64, copy=True)
        rr = np.zeros((self.K, n)) if want_rr else None
        st = np.zeros(n, dtype=np.int32)
        na = np.zeros(n, dtype=np.int32)
        nr = np.zeros(n, dtype=np.int32)
        o = opts if opts is not None else default_opts()
        if np.ndim(dt) == 0:
            dtv, dts = float(dt), None
        else:
            dtv, dts = 0.0, np.ascontiguousarray(dt, dtype=np.float64)
            assert dts.shape == (n,)
        ret = lib().orc_chem_step_dt(self._h, n, n, dtv, _dp(dts), _dp(p), _dp(T), _dp(Y), _dp(h), _dp(rr), _ip(st),
                                     _ip(na), _ip(nr), C.byref(o), int(nthreads))
        if ret < 0:
            raise ValueError("oracle chem_step: bad arguments")
        return {"T": T, "Y": Y, "h": h, "rr": rr, "status": st, "n_acc": na, "n_rej": nr}

    def rhs_v(self, rho, y):
        """Right-hand side of the constant-volume reactor at density rho."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        f = np.zeros(self.K + 1)
        lib().orc_rhs_v(self._h, float(rho), _dp(y), _dp(f))
        return f

    def jacobian_v(self, rho, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        N = self.K + 1
        J = np.zeros((N, N))
        lib().orc_jacobian_v(self._h, float(rho), _dp(y), _dp(J))
        return J

    def chem_step_v(self, T, rho, Y, dt, h_inout=None, opts=None, nthreads=0):
        """Constant-volume step of every cell: rho [n] fixed; returns dict like chem_step."""
        T = np.array(T, dtype=np.float64, copy=True)
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        Y = np.array(Y, dtype=np.float64, copy=True, order="C")
        n = T.size
        h = None if h_inout is None else np.array(h_inout, dtype=np.float64, copy=True)
        st = np.zeros(n, dtype=np.int32)
        na = np.zeros(n, dtype=np.int32)
        nr = np.zeros(n, dtype=np.int32)
        o = opts if opts is not None else default_opts()
        ret = lib().orc_chem_step_v(self._h, n, n, float(dt), _dp(rho), _dp(T), _dp(Y), _dp(h), _ip(st), _ip(na),
                                    _ip(nr), C.byref(o), int(nthreads))
        if ret < 0:
            raise ValueError("oracle chem_step_v: bad arguments")
        return {"T": T, "Y": Y, "h": h, "status": st, "n_acc": na, "n_rej": nr}

    def record(self, T, p, Y, dt, opts=None, cap=100000):
        """Integrate one cell (T, Y[K]) over dt from a fresh start; returns (T, Y, status, h_list, n_rej)
        with h_list the lengths of the accepted sub-steps."""
        y = np.concatenate([[float(T)], np.asarray(Y, dtype=np.float64)])
        hs = np.zeros(cap)
        na, nr = np.zeros(1, np.int32), np.zeros(1, np.int32)
        o = opts if opts is not None else default_opts()
        st = lib().orc_chem_cell_record(self._h, float(dt), float(p), _dp(y), C.byref(o), _dp(hs), int(cap),
                                        _ip(na), _ip(nr))
        return y[0], y[1:].copy(), int(st), hs[:min(int(na[0]), cap)].copy(), int(nr[0])

    def replay(self, p, y0, hs):
        """The fixed sequence of RODAS4 sub-steps of lengths hs from y0 = (T, Y) (no error control)."""
        y = np.array(y0, dtype=np.float64, copy=True)
        hs = np.ascontiguousarray(hs, dtype=np.float64)
        lib().orc_chem_replay(self._h, float(p), _dp(y), _dp(hs), int(hs.size))
        return y

    def scale_A(self, j, factor):
        """Multiply the pre-exponential factor of reaction j (k_inf for Troe rows) by factor, in place."""
        lib().orc_mech_scale_A(self._h, int(j), float(factor))


def rodas4_tableau():
    g = C.c_double()
    a, c = np.zeros(36), np.zeros(36)
    m, mh = np.zeros(6), np.zeros(6)
    lib().orc_rodas4_tableau(C.byref(g), _dp(a), _dp(c), _dp(m), _dp(mh))
    return g.value, a.reshape(6, 6), c.reshape(6, 6), m, mh


def linear_integrate(A, y0, dt, h_in=0.0, atol=None, **kw):
    A = np.ascontiguousarray(A, dtype=np.float64)
    y = np.array(y0, dtype=np.float64, copy=True)
    n = y.size
    at = np.full(n, 1e-12) if atol is None else np.ascontiguousarray(atol, dtype=np.float64)
    o = default_opts(**kw)
    hn = C.c_double()
    na, nr = np.zeros(1, np.int32), np.zeros(1, np.int32)
    st = lib().orc_linear_integrate(n, _dp(A), _dp(y), float(dt), float(h_in), C.byref(o), _dp(at), C.byref(hn),
                                    _ip(na), _ip(nr))
    return y, st, hn.value, int(na[0]), int(nr[0])


def linear_fixed_step(A, y0, h):
    A = np.ascontiguousarray(A, dtype=np.float64)
    y = np.array(y0, dtype=np.float64, copy=True)
    e = np.zeros_like(y)
    lib().orc_linear_fixed_step(y.size, _dp(A), _dp(y), float(h), _dp(e))
    return y, e


def bct(Y, lam):
    return lib().orc_bct(float(Y), float(lam))


def bct_inv(z, lam):
    return lib().orc_bct_inv(float(z), float(lam))


def bf16_round(x):
    return lib().orc_bf16_round(float(x))


def fp8_e4m3_round(x):
    """Nearest OCP E4M3FN value (ties to even); NaN where that exceeds 448."""
    return lib().orc_fp8_e4m3_round(float(x))


def fp8_scale_exp(amax):
    """Smallest e with amax <= 448 * 2**e (0 for amax 0)."""
    return lib().orc_fp8_scale_exp(float(amax))


class DNN:
    def __init__(self, path):
        self.path = str(path)
        self._h = lib().orc_dnn_load(self.path.encode())
        if not self._h:
            raise ValueError(f"oracle: cannot load DNN weights {path}")
        L = C.c_int()
        dims = (C.c_int * 8)()
        K = C.c_int()
        lam, dtt = C.c_double(), C.c_double()
        lib().orc_dnn_dims(self._h, C.byref(L), dims, C.byref(K), C.byref(lam), C.byref(dtt))
        self.n_layers = L.value
        self.dims = [dims[i] for i in range(L.value + 1)]
        self.K = K.value
        self.lam = lam.value
        self.dt_train = dtt.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_dnn_free(h)
            self._h = None

    def mlp(self, x_norm, mode=0):
        x = np.ascontiguousarray(x_norm, dtype=np.float64)
        u = np.zeros(self.dims[-1])
        lib().orc_mlp_forward(self._h, _dp(x), _dp(u), int(mode))
        return u

    def mlp_fp8(self, X_norm):
        """Batched forward with FP8 hidden-to-hidden layers; X_norm is n x n_in."""
        X = np.ascontiguousarray(X_norm, dtype=np.float64)
        U = np.zeros((X.shape[0], self.dims[-1]))
        lib().orc_mlp_forward_fp8(self._h, X.shape[0], _dp(X), _dp(U))
        return U

    def step(self, mech: Mech, T, p, Y, dt, renormalise=True, mode=1, fallback=True, want_rr=False, opts=None,
             nthreads=0):
        T = np.array(T, dtype=np.float64, copy=True)
        p = np.ascontiguousarray(p, dtype=np.float64)
        Y = np.array(Y, dtype=np.float64, copy=True, order="C")
        n = T.size
        rr = np.zeros((self.K, n)) if want_rr else None
        st = np.zeros(n, dtype=np.int32)
        o = opts if opts is not None else default_opts()
        ret = lib().orc_dnn_step(self._h, mech.handle, n, n, float(dt), _dp(p), _dp(T), _dp(Y), _dp(rr), _ip(st),
                                 int(renormalise), int(mode), int(fallback), C.byref(o), int(nthreads))
        if ret < 0:
            raise ValueError("oracle dnn_step: bad arguments")
        return {"T": T, "Y": Y, "rr": rr, "status": st}


def T_from_h(mech: Mech, h_target, Y, T_guess):
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    out = C.c_double()
    it = lib().orc_T_from_h(mech.handle, float(h_target), _dp(Y), float(T_guess), C.byref(out))
    return out.value, it
