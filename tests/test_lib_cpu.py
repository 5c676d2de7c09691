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
    consts = dict(re.findall(r"#define (OASIS_[A-Z0-9_]+)\s+(-?\d+(?:\.\d+)?)(?![\w.])", text))
    checked = 0
    for name, v in consts.items():
        short = name[len("OASIS_"):]
        if hasattr(L, short):
            assert getattr(L, short) == (float(v) if "." in v else int(v)), name
            checked += 1
    for short in ["OK", "EINVAL", "ENOTCONV", "ENAN", "F32", "FORM_CONV", "PSTART_ZERO", "ASSEMBLE_COLORS",
                  "KRYLOV_NULLSPACE_CONST", "MPNN_HID"]:
        assert "OASIS_" + short in consts, short
    assert checked >= 20


STRUCTS = {"oasis_csr": "Csr", "oasis_mesh": "Mesh", "oasis_krylov_opts": "KrylovOpts",
           "oasis_krylov_stats": "KrylovStats", "oasis_ipcs_params": "IpcsParams", "oasis_state": "State",
           "oasis_step_stats": "StepStats", "oasis_tuning": "Tuning", "oasis_amg_params": "AmgParams",
           "oasis_amg_level_info": "AmgLevelInfo"}


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """sizeof and every field offset of the header's structs, as the host C
    compiler lays them out, equal the ctypes declarations."""
    import shutil
    import subprocess
    from paper_1602_03643_amd import _lib as L
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "oasis.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        cls = getattr(L, pyname)
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            a, b, v = ln.split()
            got[(a, b)] = int(v)
    for cname, pyname in STRUCTS.items():
        cls = getattr(L, pyname)
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])


def test_invalid_ipcs_params_rejected_on_host(lib):
    from paper_1602_03643_amd import _lib as L
    lib = L.load()
    m = L.Mesh(3, 8, 6, 8, None, None, None, 0, None, None)
    nb = C.c_size_t()
    good = L.IpcsParams(0.01, 1e-3, (C.c_double * 3)(1, 0, 0), 0, None, 1e-8, 1e-8, 100, L.F64, 0.0, 0,
                        L.PSTART_PREV)
    assert lib.oasis_ipcs_workspace_size(C.byref(m), 40, C.byref(good), C.byref(nb)) == L.OK and nb.value > 0
    for field, bad in [("pressure_start", 7), ("precision", 5), ("dt", 0.0), ("rtol_p", -1.0),
                       ("pressure_delta", 1.5)]:
        p = L.IpcsParams.from_buffer_copy(good)
        setattr(p, field, bad)
        assert lib.oasis_ipcs_workspace_size(C.byref(m), 40, C.byref(p), C.byref(nb)) == L.EINVAL, field
    for field, bad in [("inner_iters", 17), ("velocity_update", 3), ("n_scalars", 5), ("convection", 2),
                       ("convection", -1)]:
        p = L.IpcsParams.from_buffer_copy(good)
        setattr(p, field, bad)
        assert lib.oasis_ipcs_workspace_size(C.byref(m), 40, C.byref(p), C.byref(nb)) == L.EINVAL, field
    p = L.IpcsParams.from_buffer_copy(good)
    p.n_scalars = 1
    p.diffusivity[0] = -1.0
    assert lib.oasis_ipcs_workspace_size(C.byref(m), 40, C.byref(p), C.byref(nb)) == L.EINVAL
    # storage and kernel shapes are per-call options, range-checked on the host
    for field, bad in [("storage", 9), ("grid_cap", 10), ("grid_cap", 4096), ("cg_form", -1)]:
        p = L.IpcsParams.from_buffer_copy(good)
        setattr(p.tuning, field, bad)
        assert lib.oasis_ipcs_workspace_size(C.byref(m), 40, C.byref(p), C.byref(nb)) == L.EINVAL, field


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


def test_build_script_loads_without_the_package():
    """__graft_entry__.build() must work on a fresh checkout, where the
    package refuses to import because liboasis.so is not built yet: it loads
    the build script by path, and that script imports nothing from the
    package."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import importlib.util, sys\n"
        "spec = importlib.util.spec_from_file_location('b', %r)\n"
        "m = importlib.util.module_from_spec(spec); spec.loader.exec_module(m)\n"
        "assert callable(m.build)\n"
        "assert not any(k.startswith('paper_1602_03643_amd') for k in sys.modules), sorted(sys.modules)\n"
    ) % os.path.join(root, "paper_1602_03643_amd", "build.py")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root)
    assert r.returncode == 0, r.stderr
    src = open(os.path.join(root, "__graft_entry__.py")).read()
    body = src[src.index("def build()"):src.index("def smoke()")]
    assert "spec_from_file_location" in body
    assert body.index("b.build()") < body.index("import paper_1602_03643_amd")
