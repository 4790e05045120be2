"""The C-ABI library loads and exports every entry point include/nnp.h
declares; host-side argument checks and workspace sizing (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2405_01491_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "nnp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nnp_[a-z0-9_]+)\s*\(", text)))


def test_library_built():
    assert os.path.exists(_lib.LIB_PATH), "run __graft_entry__.build() first"


def test_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared_functions()
    assert len(names) >= 22
    for name in names:
        assert hasattr(L, name), name
        assert name in _lib.SIGNATURES, name


def test_status_strings():
    L = _lib.lib()
    for code in range(10):
        assert L.nnp_status_str(code)
    assert L.nnp_status_str(2) == b"neighbour-list capacity too small"


def test_model_create_rejects_bad_arguments():
    L = _lib.lib()
    out = ctypes.c_void_p(123)
    assert L.nnp_model_create(None, None, 0, ctypes.byref(out)) == _lib.NNP_E_ARG
    shf = (ctypes.c_float * 16)(*([1.0] * 16))
    ap = _lib.AevParams(n_species=9, rc_r=5.1, n_shf_r=16, shf_r=shf, rc_a=3.5, n_shf_a=4, n_shf_z=8,
                        shf_a=shf, shf_z=shf)
    mp = _lib.MlpParams(n_layers=4)
    assert L.nnp_model_create(ctypes.byref(ap), ctypes.byref(mp), 0, ctypes.byref(out)) == _lib.NNP_E_ARG
    ap.n_species = 7
    ap.n_shf_r = 12            # the kernels are written for 16 radial shells
    assert L.nnp_model_create(ctypes.byref(ap), ctypes.byref(mp), 0, ctypes.byref(out)) == _lib.NNP_E_ARG
    ap.n_shf_r = 16
    ap.rc_a = 6.0              # angular cutoff beyond the radial one
    assert L.nnp_model_create(ctypes.byref(ap), ctypes.byref(mp), 0, ctypes.byref(out)) == _lib.NNP_E_ARG


def test_neighbors_workspace_sizing():
    L = _lib.lib()
    box = (ctypes.c_float * 3)(35.54, 35.54, 35.54)
    small = L.nnp_neighbors_workspace_bytes(4500, 1, box, ctypes.c_float(5.1))
    big = L.nnp_neighbors_workspace_bytes(99999, 1, (ctypes.c_float * 3)(99.9, 99.9, 99.9), ctypes.c_float(5.6))
    assert 0 < small < big
    # box below twice the cutoff: no valid grid
    assert L.nnp_neighbors_workspace_bytes(10, 1, (ctypes.c_float * 3)(10.0, 10.0, 10.0), ctypes.c_float(5.1)) == 0
    # open boundaries
    assert L.nnp_neighbors_workspace_bytes(72, 1, None, ctypes.c_float(5.1)) > 0


def test_md_entry_points_reject_bad_arguments():
    L = _lib.lib()
    assert L.nnp_md_kick_drift(-1, None, None, None, None, 0.5, None, None, None) == _lib.NNP_E_ARG
    assert L.nnp_md_kick(5, None, None, None, 0.5, None) == _lib.NNP_E_ARG
    assert L.nnp_md_wrap(5, None, None, None) == _lib.NNP_E_ARG
    # zero atoms is a valid no-op (nothing launched)
    assert L.nnp_md_kick(0, None, None, None, 0.5, None) == _lib.NNP_OK


@pytest.mark.parametrize("skin,every,trigger", [(0.5, 20, 1.5), (0.5, 20, 0.0), (0.5, 20, -1.0),
                                                (0.0, 5, 1.0), (0.5, 0, 1.0)])
def test_md_create_rejects_incomplete_list_settings(skin, every, trigger):
    """Settings that could let a pair come within the cutoff while missing
    from the list are refused before anything touches the device: a trigger
    outside (0, 1] with a skin, or no skin and no rebuild every step."""
    L = _lib.lib()
    buf = (ctypes.c_float * 12)()
    p = _lib.MdParams()
    p.integrator, p.dt, p.skin, p.rebuild_every, p.trigger = 0, 0.5, skin, every, trigger
    h = ctypes.c_void_p()
    dummy = ctypes.cast(buf, ctypes.c_void_p)
    st = L.nnp_md_create(dummy, 4, dummy, dummy, dummy, dummy, None, ctypes.byref(p), None, ctypes.byref(h))
    assert st == _lib.NNP_E_ARG and not h.value


@pytest.mark.parametrize("skin,every,trigger", [(0.5, 20, 1.5), (0.5, 20, 0.0), (0.0, 5, 1.0)])
def test_python_driver_rejects_incomplete_list_settings(skin, every, trigger):
    from paper_2405_01491_amd import md as nmd
    with pytest.raises(ValueError):
        nmd.VelocityVerlet(None, None, None, None, None, skin=skin, rebuild_every=every, trigger=trigger)


def test_product_path_has_no_fallback(monkeypatch, tmp_path):
    """Without the built library the binding raises instead of computing
    anything on the CPU."""
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _lib.lib()
