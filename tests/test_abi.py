"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and its host-only entry points behave."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2408_17118_amd import oica

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oica.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(oica_[a-z_0-9]+)\s*\(", src)))


def _lib():
    if not os.path.exists(oica.lib_path()):
        pytest.skip("liboica.so not built")
    return oica.load()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("oica_whiten", "oica_fixed_point", "oica_unique", "oica_create", "oica_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported():
    _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", oica.lib_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (oica_[a-z_0-9]+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    # the binding covers exactly the declared calls
    assert sorted(oica.exported_symbols()) == _declared()


def test_status_strings_and_version():
    lib = _lib()
    for code, name in oica.ERRORS.items():
        assert lib.oica_status_string(code).decode() == name
    assert lib.oica_status_string(12345).decode() == "OICA_E_UNKNOWN"
    assert lib.oica_version() >= 10000


def test_null_context_is_an_argument_error():
    lib = _lib()
    assert lib.oica_whiten(None, 4, 100, None, 0, 100, None, 1, None, None, None, None) == -1
    assert lib.oica_fixed_point(None, 4, 100, None, 1, None, 8, None, None, None, None, None,
                                None, None, None) == -1
    nu, na = C.c_int(), C.c_int()
    assert lib.oica_unique(None, 4, 100, 8, None, None, None, None, 0, None, None, None, None, None,
                           None, C.byref(nu), C.byref(na)) == -1
    assert lib.oica_create(None, 0, None) == -1
    assert lib.oica_last_error(None) == b""
    lib.oica_destroy(None)


def test_create_without_device_fails_cleanly():
    lib = _lib()
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = C.c_void_p()
    rc = lib.oica_create(C.byref(h), 0, None)
    assert rc in (-1, -5) and not h.value
