"""The C-ABI library loads and exports every function the header declares
(no compute calls: CPU only)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "fim.h")) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(fim_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("fim_create_model", "fim_set_state", "fim_get_state",
                 "fim_newton_step", "fim_solve_timestep", "fim_destroy_model",
                 "fim_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2008_01539_amd import LIB_PATH
    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_options_mirror_matches_defaults():
    """The Python options mirror carries the C defaults."""
    from paper_2008_01539_amd import fim
    c = fim._Opts()
    fim._lib.fim_default_options(ctypes.byref(c))
    py = fim.Options()
    for name, _ in fim._Opts._fields_:
        assert getattr(c, name) == getattr(py, name), name


def test_create_rejects_invalid_models_without_gpu_work():
    """Validation runs on the host before any device allocation."""
    import numpy as np
    from fimgen import make_tiny
    from paper_2008_01539_amd import FimError, FimModel
    m = make_tiny("grid3")
    bad = m.copy_with(conn_i=m.conn_j.copy(), conn_j=m.conn_i.copy())
    try:
        FimModel(bad)
        raise AssertionError("accepted conn_i > conn_j")
    except FimError as e:
        assert e.code == -1
    bad = m.copy_with(pv_ref=np.where(np.arange(m.n) == 3, 0.0, m.pv_ref))
    try:
        FimModel(bad)
        raise AssertionError("accepted zero pore volume")
    except FimError as e:
        assert e.code == -1
