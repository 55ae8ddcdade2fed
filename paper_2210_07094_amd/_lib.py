"""ctypes declarations of libdf.so (the C ABI in include/df.h)."""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdf.so")

DF_OK = 0
DF_E_INVALID = -1
DF_E_UNSUPPORTED = -2
DF_E_HIP = -3
DF_E_IO = -4
DF_E_FORMAT = -5
DF_CELL_FAILURES = 1

CELL_OK = 0
CELL_MAX_STEPS = 1
CELL_H_UNDERFLOW = 2
CELL_NONFINITE = 3
CELL_DNN_FALLBACK = 4
CELL_TAPE_FULL = 5


class ChemOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol_T", C.c_double), ("atol_Y", C.c_double), ("h_min", C.c_double),
                ("max_steps", C.c_int32), ("mapping", C.c_int32), ("schedule", C.c_int32), ("coop_blocks", C.c_int32)]


class AdamOpts(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class DnnOpts(C.Structure):
    _fields_ = [("renormalise", C.c_int32), ("fallback", C.c_int32), ("precision", C.c_int32),
                ("reserved1", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("count", C.c_int64 * 8), ("failed", C.c_int64), ("accepted", C.c_int64),
                ("rejected", C.c_int64), ("max_attempts", C.c_int32), ("max_cell", C.c_int32), ("min_Y", C.c_double)]


class DfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"df error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libdf.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2210_07094_amd.build`")
    # torch brings its own HIP runtime; it has to be initialised before the library's first HIP
    # call, or torch no longer sees the device in this process
    import torch
    if torch.cuda.is_available():
        torch.cuda.init()
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.df_last_error.restype = C.c_char_p
    L.df_last_error.argtypes = []
    L.df_version.restype = C.c_char_p
    L.df_chem_default_opts.argtypes = [C.POINTER(ChemOpts)]
    L.df_dnn_default_opts.argtypes = [C.POINTER(DnnOpts)]
    L.df_mech_load.restype = i32
    L.df_mech_load.argtypes = [C.c_char_p, i32, C.POINTER(vp)]
    L.df_mech_free.argtypes = [vp]
    L.df_mech_info.restype = i32
    L.df_mech_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    L.df_chem_workspace_size.restype = i32
    L.df_chem_workspace_size.argtypes = [vp, i64, C.POINTER(C.c_size_t)]
    L.df_chem_step.restype = i32
    L.df_chem_step.argtypes = [vp, i64, i64, d, vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, C.POINTER(ChemOpts), vp]
    L.df_chem_autotune_workspace_size.restype = i32
    L.df_chem_autotune_workspace_size.argtypes = [vp, i64, C.POINTER(C.c_size_t)]
    L.df_chem_autotune.restype = i32
    L.df_chem_autotune.argtypes = [vp, i64, i64, d, vp, vp, vp, vp, vp, C.c_size_t, C.POINTER(ChemOpts), vp]
    L.df_chem_tape_size.restype = i32
    L.df_chem_tape_size.argtypes = [vp, i64, i32, C.POINTER(C.c_size_t)]
    L.df_chem_step_taped.restype = i32
    L.df_chem_step_taped.argtypes = [vp, i64, i64, d, vp, vp, vp, vp, vp, vp, C.c_size_t, i32, C.POINTER(ChemOpts),
                                     vp]
    L.df_chem_adjoint_workspace_size.restype = i32
    L.df_chem_adjoint_workspace_size.argtypes = [vp, i64, C.POINTER(C.c_size_t)]
    L.df_chem_adjoint.restype = i32
    L.df_chem_adjoint.argtypes = [vp, i64, i64, vp, vp, C.c_size_t, i32, vp, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
    L.df_adam_default_opts.argtypes = [C.POINTER(AdamOpts)]
    L.df_dnn_trainer_create.restype = i32
    L.df_dnn_trainer_create.argtypes = [vp, i64, C.POINTER(vp)]
    L.df_dnn_trainer_free.argtypes = [vp]
    L.df_dnn_make_batch.restype = i32
    L.df_dnn_make_batch.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    L.df_dnn_train_step.restype = i32
    L.df_dnn_train_step.argtypes = [vp, i64, vp, vp, C.POINTER(AdamOpts), i32, vp, vp]
    L.df_dnn_trainer_get.restype = i32
    L.df_dnn_trainer_get.argtypes = [vp, i32, i32, vp, vp]
    L.df_dnn_trainer_set.restype = i32
    L.df_dnn_trainer_set.argtypes = [vp, i32, i32, vp, vp]
    L.df_rollout_workspace_size.restype = i32
    L.df_rollout_workspace_size.argtypes = [vp, vp, i64, C.POINTER(C.c_size_t)]
    L.df_rollout.restype = i32
    L.df_rollout.argtypes = [vp, vp, i64, i64, d, i32, i32, vp, vp, vp, vp, vp, vp, C.c_size_t, C.POINTER(ChemOpts), vp]
    L.df_chem_step_const_volume.restype = i32
    L.df_chem_step_const_volume.argtypes = [vp, i64, i64, d, vp, vp, vp, vp, vp, vp, C.POINTER(ChemOpts), vp]
    L.df_chem_step_cells.restype = i32
    L.df_chem_step_cells.argtypes = [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_size_t,
                                     C.POINTER(ChemOpts), vp]
    L.df_chem_step_noalloc.restype = i32
    L.df_chem_step_noalloc.argtypes = [vp, i64, i64, d, vp, vp, vp, vp, vp, vp, vp, C.POINTER(ChemOpts), vp]
    L.df_step_stats.restype = i32
    L.df_step_stats.argtypes = [i64, i64, i32, vp, vp, vp, vp, C.POINTER(Stats), vp]
    if hasattr(L, "df_dnn_load"):
        L.df_dnn_load.restype = i32
        L.df_dnn_load.argtypes = [C.c_char_p, vp, i32, C.POINTER(vp)]
        L.df_dnn_free.argtypes = [vp]
        L.df_dnn_info.restype = i32
        L.df_dnn_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(d), C.POINTER(d)]
        L.df_dnn_workspace_size.restype = i32
        L.df_dnn_workspace_size.argtypes = [vp, i64, C.POINTER(C.c_size_t)]
        L.df_dnn_step.restype = i32
        L.df_dnn_step.argtypes = [vp, vp, i64, i64, d, vp, vp, vp, vp, vp, vp, C.c_size_t, C.POINTER(DnnOpts),
                                  C.POINTER(ChemOpts), vp]
    _lib = L
    return L


def check(code):
    if code < 0:
        raise DfError(code, lib().df_last_error().decode(errors="replace"))
    return code


def header_symbols(header_path=None):
    """Function names declared in include/df.h."""
    import re
    if header_path is None:
        header_path = os.path.join(os.path.dirname(PKG), "include", "df.h")
    txt = open(header_path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(df_[a-z_0-9]+)\s*\(", txt)))
