"""The C-ABI library loads and exports every entry point that include/*.h
declares; argument checks that need no device run on the CPU."""
import ctypes
import glob
import os
import re

import pytest

from paper_2407_00041_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\([^;{]*\)\s*;", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_abi():
    names = declared_functions()
    for n in ["dirac_create", "dirac_destroy", "dirac_apply", "dirac_apply_adjoint", "dirac_apply_batched",
              "dirac_pack", "dirac_unpack", "fgmres_solve", "fgmres_workspace_bytes", "dirac_force",
              "dirac_force_workspace_bytes", "dirac_clover_term", "dirac_last_error"]:
        assert n in names


def test_header_constants_match_binding():
    """Every status code, precision, flag and solver mode the header defines
    has the same value in the Python binding; the solver parameter record has
    the header's fields in order."""
    text = open(os.path.join(ROOT, "include", "wdirac.h")).read()
    defs = dict(re.findall(r"^#define (WDIRAC_\w+|FGMRES_\w+)\s+\(?(-?\d+)u?\)?", text, flags=re.M))
    assert len(defs) >= 18
    for name, value in defs.items():
        attr = name[len("WDIRAC_"):] if name.startswith("WDIRAC_") else name
        assert getattr(_lib, attr) == int(value), name
    end = text.index("} fgmres_params;")
    body = text[text.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"(\w+)\s*;", body)
    assert fields == [f[0] for f in _lib.FgmresParams._fields_]


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(_lib.SIGNATURES) >= declared_functions()


def test_argument_errors_without_device():
    lib = _lib.load()
    assert lib.dirac_apply(None, None, None, 1, 0, None) == _lib.EINVAL
    assert b"null" in lib.dirac_last_error()
    assert lib.dirac_apply_adjoint(None, None, None, 1, 0, None) == _lib.EINVAL
    h = ctypes.c_void_p()
    bad = (ctypes.c_int * 4)(4, 4, 1, 4)
    assert lib.dirac_create(ctypes.byref(h), bad, ctypes.c_void_p(1), None, 0.0, 0.0, 0) == _lib.EINVAL
    assert h.value is None
    assert lib.dirac_create(None, bad, None, None, 0.0, 0.0, 0) == _lib.EINVAL
    assert lib.dirac_destroy(None) == 0
    assert lib.dirac_volume(None) == 0
    assert lib.dirac_field_bytes(None, 0, 1) == 0
    assert lib.dirac_pack(None, None, None, 1, 0, None) == _lib.EINVAL
    assert lib.dirac_clover_term(None, None, None, None) == _lib.EINVAL
    # even-odd entry points and the force: a null operator is rejected before any device call
    assert lib.dirac_parity_field_bytes(None, 0, 1) == 0
    assert lib.dirac_parity_split(None, None, None, None, 1, 0, None) == _lib.EINVAL
    assert lib.dirac_parity_merge(None, None, None, None, 1, 0, None) == _lib.EINVAL
    assert lib.dirac_apply_schur(None, None, None, None, 1, 0, 0, None) == _lib.EINVAL
    assert lib.dirac_schur_prepare(None, None, None, None, None, 1, 0, None) == _lib.EINVAL
    assert lib.dirac_schur_reconstruct(None, None, None, None, 1, 0, None) == _lib.EINVAL
    assert b"null operator" in lib.dirac_last_error()
    assert lib.dirac_force_workspace_bytes(None) == 0
    assert lib.dirac_force(None, None, None, None, 1, 0, None, 0, None) == _lib.EINVAL


def test_product_path_has_no_fallback(monkeypatch, tmp_path):
    """Without the shared object the binding raises instead of computing."""
    monkeypatch.setattr(_lib, "SO_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.load()
