"""The C ABI library: it loads, exports every function df.h declares, and
rejects bad arguments on the host before touching the GPU (CPU-only checks)."""
import ctypes as C
import os

import pytest

import paper_2210_07094_amd as df
from paper_2210_07094_amd import _lib


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libdf.so is not built: run `python -m paper_2210_07094_amd.build`")
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _lib.header_symbols()
    assert "df_chem_step" in names and "df_mech_load" in names and "df_dnn_step" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_default_opts(L):
    o = df.chem_opts()
    assert (o.rtol, o.atol_T, o.atol_Y, o.h_min, o.max_steps, o.mapping) == (1e-8, 1e-6, 1e-14, 1e-20, 100000, 0)
    assert (o.schedule, o.coop_blocks) == (0, 0)
    d = df.dnn_opts()
    assert (d.renormalise, d.fallback) == (1, 1)


def test_mech_load_errors(L, tmp_path):
    h = C.c_void_p()
    assert L.df_mech_load(None, 0, C.byref(h)) == _lib.DF_E_INVALID
    assert L.df_mech_load(b"/nonexistent/file.mech", 0, C.byref(h)) == _lib.DF_E_IO
    assert b"cannot open" in L.df_last_error()
    bad = tmp_path / "bad.mech"
    bad.write_text("dfmech 1\nname x\nseed 0\nn_elements 1\nn_species 2\nn_reactions 0\nelements X\nelement_mass 1\n"
                   "species A B\nmolar_mass 1 -2\n")
    assert L.df_mech_load(str(bad).encode(), 0, C.byref(h)) == _lib.DF_E_FORMAT


def test_chem_step_host_checks(L):
    o = df.chem_opts()
    assert L.df_chem_step(None, 1, 1, 1e-6, None, None, None, None, None, None, None, None, 0, C.byref(o), None) \
        == _lib.DF_E_INVALID
    assert b"null mechanism" in L.df_last_error()


def test_chem_step_cells_and_autotune_host_checks(L):
    o = df.chem_opts()
    # per-cell step lengths: a null dt array is refused before anything else
    assert L.df_chem_step_cells(None, 1, 1, None, None, None, None, None, None, None, None, None, 0, C.byref(o),
                                None) == _lib.DF_E_INVALID
    assert b"null dt" in L.df_last_error()
    b = C.c_size_t()
    assert L.df_chem_autotune_workspace_size(None, 1, C.byref(b)) == _lib.DF_E_INVALID
    assert L.df_chem_autotune(None, 1, 1, 1e-6, None, None, None, None, None, 0, C.byref(o), None) \
        == _lib.DF_E_INVALID
    assert L.df_chem_autotune(None, 1, 1, 1e-6, None, None, None, None, None, 0, None, None) == _lib.DF_E_INVALID


def test_dnn_step_host_checks(L):
    assert L.df_dnn_step(None, None, 1, 1, 1e-6, None, None, None, None, None, None, 0, None, None, None) \
        == _lib.DF_E_INVALID


def test_binding_refuses_cpu_tensors(L):
    import torch
    with pytest.raises(ValueError):
        df._ptr(torch.zeros(3, dtype=torch.float64), torch.float64, "T")


def test_adjoint_host_checks(L):
    o = df.chem_opts()
    b = C.c_size_t()
    assert L.df_chem_tape_size(None, 1, 10, C.byref(b)) == _lib.DF_E_INVALID
    assert L.df_chem_adjoint_workspace_size(None, 1, C.byref(b)) == _lib.DF_E_INVALID
    assert L.df_chem_step_taped(None, 1, 1, 1e-6, None, None, None, None, None, None, 0, 10, C.byref(o), None) \
        == _lib.DF_E_INVALID
    assert b"null mechanism" in L.df_last_error()
    assert L.df_chem_adjoint(None, 1, 1, None, None, 0, 10, None, None, None, None, None, None, None, 0, None) \
        == _lib.DF_E_INVALID
    assert b"null mechanism" in L.df_last_error()


def test_const_volume_and_rollout_host_checks(L):
    o = df.chem_opts()
    assert L.df_chem_step_const_volume(None, 1, 1, 1e-6, None, None, None, None, None, None, C.byref(o), None) \
        == _lib.DF_E_INVALID
    assert b"null mechanism" in L.df_last_error()
    b = C.c_size_t()
    assert L.df_rollout_workspace_size(None, None, 1, C.byref(b)) == _lib.DF_E_INVALID
    assert L.df_rollout(None, None, 1, 1, 1e-6, 10, 0, None, None, None, None, None, None, 0, None, None) \
        == _lib.DF_E_INVALID
    assert b"null mechanism" in L.df_last_error()


def test_step_stats_host_checks(L):
    s = _lib.Stats()
    # null device summary, negative cell count, Y without species count: refused before any launch
    assert L.df_step_stats(4, 4, 0, None, None, None, None, C.byref(s), None) == _lib.DF_E_INVALID
    assert b"null stats_dev" in L.df_last_error()
    fake = C.c_void_p(4096)   # never dereferenced: the argument checks come first
    assert L.df_step_stats(-1, 4, 0, None, None, None, fake, C.byref(s), None) == _lib.DF_E_INVALID
    assert L.df_step_stats(4, 4, 0, None, None, fake, fake, C.byref(s), None) == _lib.DF_E_INVALID
    assert L.df_step_stats(4, 2, 9, None, None, fake, fake, C.byref(s), None) == _lib.DF_E_INVALID
    assert L.df_step_stats(4, 4, 0, None, None, None, C.c_void_p(4097), C.byref(s), None) == _lib.DF_E_INVALID
    assert b"aligned" in L.df_last_error()
    assert C.sizeof(_lib.Stats) == 8 * 12 + 8 + 8
