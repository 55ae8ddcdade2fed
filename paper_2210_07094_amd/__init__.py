"""Per-cell chemistry step on MI355X (gfx950): Python binding of libdf.so.

Every step of the computation runs in the HIP library; this module only
passes torch tensors (device memory) and the current HIP stream through the
C ABI declared in ``include/df.h``.

    import paper_2210_07094_amd as df
    mech = df.Mechanism("synth/data/h2_synth_9sp_24r.mech")
    st = mech.chem_step(T, p, Y, 1e-6)        # T[n], p[n], Y[K, ld] float64 cuda tensors, in place
"""
from __future__ import annotations

import ctypes as C

from ._lib import (CELL_DNN_FALLBACK, CELL_H_UNDERFLOW, CELL_MAX_STEPS, CELL_NONFINITE, CELL_OK,  # noqa
                   CELL_TAPE_FULL, DF_CELL_FAILURES, AdamOpts, ChemOpts, DfError, DnnOpts, Stats, check, lib)

__all__ = ["Mechanism", "DNN", "Trainer", "chem_opts", "dnn_opts", "adam_opts", "chem_step_diff", "step_stats",
           "DfError", "lib"]


def chem_opts(**kw) -> ChemOpts:
    o = ChemOpts()
    lib().df_chem_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def dnn_opts(**kw) -> DnnOpts:
    o = DnnOpts()
    lib().df_dnn_default_opts(C.byref(o))
    names = {f[0] for f in DnnOpts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"dnn_opts: unknown option {k!r}")
        setattr(o, k, v)
    return o


def adam_opts(**kw) -> AdamOpts:
    o = AdamOpts()
    lib().df_adam_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(t, dtype, name, numel=None, device=None):
    """data pointer of a contiguous cuda tensor of the given dtype (None passes NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: expected a device (cuda/HIP) tensor, got {t.device}")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name}: tensor on device {t.device.index}, handle on device {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: needs at least {numel} elements, has {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def step_stats(n_cells, status=None, n_steps=None, Y=None, stats_dev=None, stream=None):
    """Summary of a finished step (df_step_stats) from its per-cell outputs: status int32 [n],
    n_steps int32 [2n], Y float64 [K, ld] device tensors (each optional).  Waits for the stream and
    returns (failures, summary): failures is True when df_step_stats returned DF_CELL_FAILURES,
    summary a dict of the df_stats fields (count as a list per status code).  stats_dev: a device
    uint8 tensor of at least sizeof(df_stats) bytes to hold the device copy (allocated if None)."""
    import torch
    n = int(n_cells)
    size = C.sizeof(Stats)
    if stats_dev is None:
        dev = next((t.device for t in (status, n_steps, Y) if t is not None), torch.device("cuda"))
        stats_dev = torch.empty(size, dtype=torch.uint8, device=dev)
    if stats_dev.dtype != torch.uint8 or stats_dev.numel() < size:
        raise ValueError(f"stats_dev: needs a uint8 device tensor of at least {size} bytes")
    K, ld = (0, n) if Y is None else (int(Y.shape[0]), int(Y.shape[1]))
    host = Stats()
    code = check(lib().df_step_stats(n, ld, K, _ptr(status, torch.int32, "status", n),
                                     _ptr(n_steps, torch.int32, "n_steps", 2 * n),
                                     _ptr(Y, torch.float64, "Y", K * ld), C.c_void_p(stats_dev.data_ptr()),
                                     C.byref(host), _stream(stream)))
    out = {f[0]: getattr(host, f[0]) for f in Stats._fields_}
    out["count"] = list(host.count)
    return code == DF_CELL_FAILURES, out


class Mechanism:
    """A loaded mechanism (df_mech_load); tables live on `device`."""

    def __init__(self, path, device: int = 0):
        self.path = str(path)
        self.device = int(device)
        h = C.c_void_p()
        check(lib().df_mech_load(self.path.encode(), self.device, C.byref(h)))
        self._h = h
        K, M, E = C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().df_mech_info(self._h, C.byref(K), C.byref(M), C.byref(E)))
        self.n_species, self.n_reactions, self.n_elements = K.value, M.value, E.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().df_mech_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, n_cells: int) -> int:
        b = C.c_size_t()
        check(lib().df_chem_workspace_size(self._h, int(n_cells), C.byref(b)))
        return b.value

    def workspace(self, n_cells: int):
        import torch
        return torch.empty(max(self.workspace_bytes(n_cells), 1), dtype=torch.uint8, device=f"cuda:{self.device}")

    def chem_step(self, T, p, Y, dt, h=None, rr=None, status=None, n_steps=None, workspace=None, opts=None,
                  stream=None):
        """Advance every cell by dt in place (df_chem_step, or df_chem_step_cells when dt is a
        float64 device tensor [n] of per-cell step lengths).

        T, p: float64 [n]; Y: float64 [K, ld] (species-major, ld >= n); optional
        h [n] (sub-step hint, in/out), rr [K, ld], status int32 [n], n_steps
        int32 [2n], workspace uint8 (cost ordering and the queue schedule; see
        workspace()).  Asynchronous on `stream` (default: torch's current stream).
        """
        import torch
        n = T.numel()
        K = self.n_species
        if Y.dim() != 2 or Y.shape[0] != K:
            raise ValueError(f"Y must have shape [{K}, ld]")
        ld = Y.shape[1]
        dev = self.device
        per_cell = isinstance(dt, torch.Tensor)
        dt_arg = _ptr(dt, torch.float64, "dt", n, dev) if per_cell else float(dt)
        args = (self._h, n, ld, dt_arg,
                _ptr(p, torch.float64, "p", n, dev), _ptr(T, torch.float64, "T", n, dev),
                _ptr(Y, torch.float64, "Y", K * ld, dev), _ptr(h, torch.float64, "h", n, dev),
                _ptr(rr, torch.float64, "rr", K * ld, dev), _ptr(status, torch.int32, "status", n, dev),
                _ptr(n_steps, torch.int32, "n_steps", 2 * n, dev),
                _ptr(workspace, torch.uint8, "workspace", None, dev), 0 if workspace is None else workspace.numel(),
                C.byref(opts) if opts is not None else None, _stream(stream))
        return check(lib().df_chem_step_cells(*args) if per_cell else lib().df_chem_step(*args))


    def chem_step_const_volume(self, T, rho, Y, dt, h=None, status=None, n_steps=None, opts=None, stream=None):
        """Advance every cell by dt at constant volume, in place (df_chem_step_const_volume):
        rho float64 [n] densities, other arguments as chem_step."""
        import torch
        n = T.numel()
        K = self.n_species
        if Y.dim() != 2 or Y.shape[0] != K:
            raise ValueError(f"Y must have shape [{K}, ld]")
        ld = Y.shape[1]
        dev = self.device
        return check(lib().df_chem_step_const_volume(
            self._h, n, ld, float(dt), _ptr(rho, torch.float64, "rho", n, dev), _ptr(T, torch.float64, "T", n, dev),
            _ptr(Y, torch.float64, "Y", K * ld, dev), _ptr(h, torch.float64, "h", n, dev),
            _ptr(status, torch.int32, "status", n, dev), _ptr(n_steps, torch.int32, "n_steps", 2 * n, dev),
            C.byref(opts) if opts is not None else None, _stream(stream)))

    def rollout(self, T, p, Y, dt, n_steps, dnn=None, trajectory=False, constant_volume=False, opts=None,
                stream=None):
        """n_steps consecutive steps of the DNN (dnn given) or of the integrator on (T, Y) in place,
        with each cell's ignition delay (df_rollout).  With constant_volume the integrator steps the
        constant-volume reactor and p holds the density.  Returns (idt [n], T_traj [n_steps+1, n]
        or None)."""
        import torch
        n = T.numel()
        K = self.n_species
        if Y.dim() != 2 or Y.shape[0] != K:
            raise ValueError(f"Y must have shape [{K}, ld]")
        ld = Y.shape[1]
        dev = self.device
        dh = dnn.handle if dnn is not None else None
        b = C.c_size_t()
        check(lib().df_rollout_workspace_size(self._h, dh, n, C.byref(b)))
        ws = torch.empty(max(b.value, 1), dtype=torch.uint8, device=f"cuda:{dev}")
        idt = torch.empty(n, dtype=torch.float64, device=f"cuda:{dev}")
        traj = torch.empty(int(n_steps) + 1, n, dtype=torch.float64, device=f"cuda:{dev}") if trajectory else None
        check(lib().df_rollout(self._h, dh, n, ld, float(dt), int(n_steps), 1 if constant_volume else 0,
                               _ptr(p, torch.float64, "p", n, dev),
                               _ptr(T, torch.float64, "T", n, dev), _ptr(Y, torch.float64, "Y", K * ld, dev),
                               _ptr(idt, torch.float64, "idt", n, dev),
                               _ptr(traj, torch.float64, "T_traj", None, dev), _ptr(ws, torch.uint8, "ws", None, dev),
                               ws.numel(), C.byref(opts) if opts is not None else None, _stream(stream)))
        return idt, traj

    def autotune(self, T, p, Y, dt, opts=None, stream=None) -> ChemOpts:
        """Schedule for this workload (df_chem_autotune): times the candidates on copies of
        (T, Y) and returns `opts` (or the defaults) with schedule and coop_blocks set."""
        import torch
        n = T.numel()
        K = self.n_species
        if Y.dim() != 2 or Y.shape[0] != K:
            raise ValueError(f"Y must have shape [{K}, ld]")
        ld = Y.shape[1]
        dev = self.device
        o = ChemOpts()
        if opts is None:
            lib().df_chem_default_opts(C.byref(o))
        else:
            C.pointer(o)[0] = opts
        b = C.c_size_t()
        check(lib().df_chem_autotune_workspace_size(self._h, n, C.byref(b)))
        ws = torch.empty(max(b.value, 1), dtype=torch.uint8, device=f"cuda:{dev}")
        per_cell = isinstance(dt, torch.Tensor)
        check(lib().df_chem_autotune(self._h, n, ld, 0.0 if per_cell else float(dt),
                                     _ptr(dt, torch.float64, "dt", n, dev) if per_cell else None,
                                     _ptr(p, torch.float64, "p", n, dev), _ptr(T, torch.float64, "T", n, dev),
                                     _ptr(Y, torch.float64, "Y", K * ld, dev), _ptr(ws, torch.uint8, "ws", None, dev),
                                     ws.numel(), C.byref(o), _stream(stream)))
        return o

    # ---- discrete adjoint (df_chem_step_taped / df_chem_adjoint)

    def tape_bytes(self, n_cells: int, max_substeps: int) -> int:
        b = C.c_size_t()
        check(lib().df_chem_tape_size(self._h, int(n_cells), int(max_substeps), C.byref(b)))
        return b.value

    def chem_step_taped(self, T, p, Y, dt, max_substeps=1024, status=None, n_steps=None, opts=None, stream=None):
        """df_chem_step (each cell from a fresh start) that records the adjoint's tape; T, Y in
        place.  Returns the tape (uint8 device tensor) for chem_adjoint."""
        import torch
        n = T.numel()
        K = self.n_species
        if Y.dim() != 2 or Y.shape[0] != K:
            raise ValueError(f"Y must have shape [{K}, ld]")
        ld = Y.shape[1]
        dev = self.device
        tape = torch.empty(max(self.tape_bytes(n, max_substeps), 1), dtype=torch.uint8, device=f"cuda:{dev}")
        check(lib().df_chem_step_taped(self._h, n, ld, float(dt), _ptr(p, torch.float64, "p", n, dev),
                                       _ptr(T, torch.float64, "T", n, dev), _ptr(Y, torch.float64, "Y", K * ld, dev),
                                       _ptr(status, torch.int32, "status", n, dev),
                                       _ptr(n_steps, torch.int32, "n_steps", 2 * n, dev),
                                       _ptr(tape, torch.uint8, "tape", None, dev), tape.numel(), int(max_substeps),
                                       C.byref(opts) if opts is not None else None, _stream(stream)))
        return tape

    def chem_adjoint(self, p, tape, max_substeps, T_bar, Y_bar, per_cell=True, summed=True, stream=None):
        """Reverse sweep over a tape (df_chem_adjoint).  T_bar [n], Y_bar [K, ld] seeds.  Returns
        (T0_bar [n], Y0_bar [K, ld], lnA_bar_cells [M, ld] or None, lnA_bar [M] or None)."""
        import torch
        n = T_bar.numel()
        K, M = self.n_species, self.n_reactions
        if Y_bar.dim() != 2 or Y_bar.shape[0] != K:
            raise ValueError(f"Y_bar must have shape [{K}, ld]")
        ld = Y_bar.shape[1]
        dev = self.device
        opt = dict(dtype=torch.float64, device=f"cuda:{dev}")
        T0b = torch.empty(n, **opt)
        Y0b = torch.empty(K, ld, **opt)
        thc = torch.empty(M, ld, **opt) if per_cell else None
        ths = torch.empty(M, **opt) if summed else None
        b = C.c_size_t()
        check(lib().df_chem_adjoint_workspace_size(self._h, n, C.byref(b)))
        ws = torch.empty(max(b.value, 1), dtype=torch.uint8, device=f"cuda:{dev}")
        check(lib().df_chem_adjoint(self._h, n, ld, _ptr(p, torch.float64, "p", n, dev),
                                    _ptr(tape, torch.uint8, "tape", None, dev), tape.numel(), int(max_substeps),
                                    _ptr(T_bar, torch.float64, "T_bar", n, dev),
                                    _ptr(Y_bar, torch.float64, "Y_bar", K * ld, dev),
                                    _ptr(T0b, torch.float64, "T0_bar", n, dev),
                                    _ptr(Y0b, torch.float64, "Y0_bar", K * ld, dev),
                                    _ptr(thc, torch.float64, "lnA_bar_cells", M * ld, dev),
                                    _ptr(ths, torch.float64, "lnA_bar", M, dev),
                                    _ptr(ws, torch.uint8, "workspace", None, dev), ws.numel(), _stream(stream)))
        return T0b, Y0b, thc, ths


def _chem_step_function():
    import torch

    class ChemStepFunction(torch.autograd.Function):
        """(T0, Y0, lnA) -> (T, Y) after one chemistry step; backward = the discrete adjoint."""

        @staticmethod
        def forward(ctx, T0, Y0, lnA, mech, p, dt, max_substeps, opts):
            T = T0.detach().clone()
            Y = Y0.detach().contiguous().clone()
            status = torch.empty(T.numel(), dtype=torch.int32, device=T.device)
            tape = mech.chem_step_taped(T, p, Y, dt, max_substeps=max_substeps, status=status, opts=opts)
            ctx.mech, ctx.max_substeps = mech, max_substeps
            ctx.save_for_backward(p, tape)
            ctx.status = status
            return T, Y

        @staticmethod
        def backward(ctx, gT, gY):
            p, tape = ctx.saved_tensors
            mech = ctx.mech
            n = p.numel()
            gT = torch.zeros(n, dtype=torch.float64, device=p.device) if gT is None else gT.contiguous()
            gY = (torch.zeros(mech.n_species, n, dtype=torch.float64, device=p.device) if gY is None
                  else gY.contiguous())
            want_lnA = ctx.needs_input_grad[2]
            T0b, Y0b, _, lnAb = mech.chem_adjoint(p, tape, ctx.max_substeps, gT, gY, per_cell=False, summed=want_lnA)
            return T0b, Y0b, lnAb, None, None, None, None, None

    return ChemStepFunction


_ChemStepFunction = None


def chem_step_diff(mech: Mechanism, T0, Y0, p, dt, lnA=None, max_substeps=1024, opts=None):
    """Differentiable chemistry step: returns (T, Y) after dt, with gradients to T0 [n], Y0 [K, n]
    and, when lnA is given, to it.  lnA is a float64 device tensor [M] standing for the natural
    logs of the mechanism's pre-exponential factors (k_inf's for falloff rows) in the file's
    reaction order; the step uses the loaded mechanism, so lnA only receives d loss / d ln A
    (summed over cells).  Backward runs df_chem_adjoint over the tape of the forward step; cells
    whose step failed or overflowed max_substeps get zero gradients (Mechanism.chem_step_taped
    reports the per-cell status)."""
    global _ChemStepFunction
    import torch
    if _ChemStepFunction is None:
        _ChemStepFunction = _chem_step_function()
    if lnA is None:
        lnA = torch.zeros(mech.n_reactions, dtype=torch.float64, device=T0.device)
    return _ChemStepFunction.apply(T0, Y0, lnA, mech, p, dt, max_substeps, opts)


class DNN:
    """A loaded DNN chemistry integrator (df_dnn_load)."""

    def __init__(self, path, mech: Mechanism, device: int = 0):
        self.path = str(path)
        self.mech = mech
        self.device = int(device)
        h = C.c_void_p()
        check(lib().df_dnn_load(self.path.encode(), mech.handle, self.device, C.byref(h)))
        self._h = h
        L = C.c_int32()
        dims = (C.c_int32 * 16)()
        lam, dtt = C.c_double(), C.c_double()
        check(lib().df_dnn_info(self._h, C.byref(L), dims, C.byref(lam), C.byref(dtt)))
        self.n_layers = L.value
        self.dims = [dims[i] for i in range(L.value + 1)]
        self.lam = lam.value
        self.dt_train = dtt.value
        self.K = self.dims[-1]

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().df_dnn_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, n_cells: int) -> int:
        b = C.c_size_t()
        check(lib().df_dnn_workspace_size(self._h, int(n_cells), C.byref(b)))
        return b.value

    def workspace(self, n_cells: int):
        import torch
        nb = self.workspace_bytes(n_cells)
        return torch.empty(max(nb, 1), dtype=torch.uint8, device=f"cuda:{self.device}")

    def step(self, T, p, Y, dt, rr=None, status=None, workspace=None, opts=None, fallback_opts=None, stream=None):
        """DNN chemistry step in place (df_dnn_step); arguments as Mechanism.chem_step."""
        import torch
        n = T.numel()
        K = self.mech.n_species
        if Y.dim() != 2 or Y.shape[0] != K:
            raise ValueError(f"Y must have shape [{K}, ld]")
        ld = Y.shape[1]
        dev = self.device
        if workspace is None:
            workspace = self.workspace(n)
        if workspace.dtype != torch.uint8:
            raise TypeError("workspace must be a uint8 tensor")
        args = (self._h, self.mech.handle, n, ld, float(dt),
                _ptr(p, torch.float64, "p", n, dev), _ptr(T, torch.float64, "T", n, dev),
                _ptr(Y, torch.float64, "Y", K * ld, dev), _ptr(rr, torch.float64, "rr", K * ld, dev),
                _ptr(status, torch.int32, "status", n, dev), _ptr(workspace, torch.uint8, "workspace", None, dev),
                workspace.numel(), C.byref(opts) if opts is not None else None,
                C.byref(fallback_opts) if fallback_opts is not None else None, _stream(stream))
        return check(lib().df_dnn_step(*args))


class Trainer:
    """Training state of a DNN handle on its device (df_dnn_trainer_create); each update rewrites
    the handle's weights."""

    def __init__(self, dnn: "DNN", max_batch: int):
        self.dnn = dnn
        self.max_batch = int(max_batch)
        h = C.c_void_p()
        check(lib().df_dnn_trainer_create(dnn.handle, self.max_batch, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().df_dnn_trainer_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def make_batch(self, p, T, Y0, Y1, stream=None):
        """(x [n, K+2], target [n, K], valid [n]) from states before (p, T, Y0) and after (Y1) an
        integrator step of the network's dt (df_dnn_make_batch)."""
        import torch
        n = T.numel()
        K = self.dnn.K
        dev = self.dnn.device
        ld = Y0.shape[1]
        x = torch.empty(n, K + 2, dtype=torch.float32, device=f"cuda:{dev}")
        t = torch.empty(n, K, dtype=torch.float32, device=f"cuda:{dev}")
        v = torch.empty(n, dtype=torch.int32, device=f"cuda:{dev}")
        check(lib().df_dnn_make_batch(self.dnn.handle, n, ld, _ptr(p, torch.float64, "p", n, dev),
                                      _ptr(T, torch.float64, "T", n, dev), _ptr(Y0, torch.float64, "Y0", K * ld, dev),
                                      _ptr(Y1, torch.float64, "Y1", K * ld, dev), _ptr(x, torch.float32, "x"),
                                      _ptr(t, torch.float32, "target"), _ptr(v, torch.int32, "valid"),
                                      _stream(stream)))
        return x, t, v

    def step(self, x, target, opts=None, update=True, stream=None):
        """One training step on the rows of x [B, K+2], target [B, K] (fp32 device); returns the
        loss before the update as a 1-element device tensor."""
        import torch
        dev = self.dnn.device
        B = x.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device=f"cuda:{dev}")
        check(lib().df_dnn_train_step(self._h, B, _ptr(x, torch.float32, "x", B * x.shape[1], dev),
                                      _ptr(target, torch.float32, "target", B * target.shape[1], dev),
                                      C.byref(opts) if opts is not None else None, 1 if update else 0,
                                      _ptr(loss, torch.float32, "loss", 1, dev), _stream(stream)))
        return loss

    def get(self, layer: int, what: str, stream=None):
        """'W', 'b', 'dW' or 'db' of layer `layer` (fp32 device tensor, unpadded)."""
        import torch
        code = {"W": 0, "b": 1, "dW": 2, "db": 3}[what]
        dims = self.dnn.dims
        shape = (dims[layer + 1], dims[layer]) if code in (0, 2) else (dims[layer + 1],)
        out = torch.empty(*shape, dtype=torch.float32, device=f"cuda:{self.dnn.device}")
        check(lib().df_dnn_trainer_get(self._h, int(layer), code, _ptr(out, torch.float32, what), _stream(stream)))
        return out

    def set(self, layer: int, what: str, value, stream=None):
        """Set 'W' [n_out, n_in] or 'b' [n_out] of layer `layer` (fp32 device tensor)."""
        import torch
        code = {"W": 0, "b": 1}[what]
        dims = self.dnn.dims
        numel = dims[layer + 1] * dims[layer] if code == 0 else dims[layer + 1]
        check(lib().df_dnn_trainer_set(self._h, int(layer), code,
                                       _ptr(value, torch.float32, what, numel, self.dnn.device), _stream(stream)))
