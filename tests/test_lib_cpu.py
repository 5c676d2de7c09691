"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every function declared in include/oasis.h, and rejects invalid arguments
before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oasis.h")
LIB = os.path.join(ROOT, "paper_1602_03643_amd", "liboasis.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(oasis_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liboasis.so not built; run __graft_entry__.build()")
    return C.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1602_03643_amd import _lib as L
    assert set(_declared()) == set(L._SIGS)


def test_header_constants_match_binding():
    from paper_1602_03643_amd import _lib as L
    text = open(HEADER).read()
    consts = dict(re.findall(r"#define (OASIS_[A-Z0-9_]+)\s+(-?\d+)\b", text))
    assert int(consts["OASIS_OK"]) == L.OK and int(consts["OASIS_EINVAL"]) == L.EINVAL
    assert int(consts["OASIS_ENOTCONV"]) == L.ENOTCONV and int(consts["OASIS_ENAN"]) == L.ENAN
    assert int(consts["OASIS_FORM_CONV"]) == L.FORM_CONV and int(consts["OASIS_F32"]) == L.F32


def test_invalid_arguments_rejected_on_host(lib):
    from paper_1602_03643_amd import _lib as L
    lib = L.load()
    assert lib.oasis_spmv(None, None, None, None, 1.0, 0.0) == L.EINVAL
    bad = L.Csr(0, 0, None, None, None, L.F64)
    assert lib.oasis_spmv(None, C.byref(bad), None, None, 1.0, 0.0) == L.EINVAL
    nb = C.c_size_t()
    assert lib.oasis_krylov_workspace_size(10, 30, 4, None, C.byref(nb)) == L.EINVAL
    o = L.KrylovOpts(1e-8, 100, 0, 1e-4, 10, 0, 0)
    assert lib.oasis_krylov_workspace_size(10, 30, 3, C.byref(o), C.byref(nb)) == L.OK and nb.value > 0
    m = L.Mesh(4, 10, 10, 10, None, None, None, 0, None, None)
    assert lib.oasis_graph_workspace_size(C.byref(m), C.byref(nb)) == L.EINVAL
    assert lib.oasis_strerror(L.ENOTCONV).decode().startswith("Krylov")
    assert b"gfx950" in lib.oasis_version()
