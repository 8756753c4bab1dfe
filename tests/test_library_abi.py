"""The C-ABI library loads and exports every entry point include/lp.h
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lp_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2206_14061_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2206_14061_amd import build
        build.build(verbose=False)
    return _lib.LIB_PATH


def test_header_declares_the_six_method_entry_points():
    names = _declared()
    for n in ("lp_build_cells", "lp_neighbors", "lp_fit_derivs",
              "lp_rheology_rhs", "lp_step", "lp_step_adjoint"):
        assert n in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    from paper_2206_14061_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared()


def test_struct_layouts_match_header():
    """ctypes mirrors of lp_params / lp_config / lp_state have the C sizes
    (20 doubles; natural alignment; 7 pointers)."""
    from paper_2206_14061_amd import _lib
    assert ctypes.sizeof(_lib.LPParams) == 20 * 8
    assert ctypes.sizeof(_lib.LPConfig) == 72
    assert _lib.LPConfig.min_real_rows.offset == 68
    assert ctypes.sizeof(_lib.LPState) == 7 * 8
    # lp_step_record: force_sort, resorted (int32), list_gen (int64), perm
    assert ctypes.sizeof(_lib.LPStepRecord) == 24
    assert _lib.LPStepRecord.list_gen.offset == 8
    assert _lib.LPStepRecord.perm.offset == 16


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2206_14061_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        _lib.load()


def test_enum_constants_match_header():
    """Every LP_* enum constant of include/lp.h has the same value in the
    binding (debug flags, precision, weights)."""
    from paper_2206_14061_amd import _lib
    text = open(os.path.join(ROOT, "include", "lp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    found = 0
    for body in re.findall(r"enum\s*\{([^}]*)\}", text):
        for name, val in re.findall(r"(LP_[A-Z0-9_]+)\s*=\s*(\d+)", body):
            assert getattr(_lib, name) == int(val), name
            found += 1
    assert found >= 12
    assert _lib.LP_DEBUG_PARTICLE_LIST == 128
