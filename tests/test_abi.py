"""CPU checks of the C ABI library: it loads and exports every declared
symbol; no compute calls (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcrt.h")
LIB = os.path.join(ROOT, "paper_2110_15640_amd", "libmcrt.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mcrt_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["mcrt_grid_upload", "mcrt_opacity_upload", "mcrt_solve_albedo", "mcrt_solve_emission",
              "mcrt_solve_transmission", "mcrt_create", "mcrt_destroy", "mcrt_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcrt.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcrt.so not built")
def test_binding_struct_layouts_match_header():
    """The ctypes structs must mirror the C structs field by field."""
    from paper_2110_15640_amd import mcrt as M
    txt = open(HEADER).read()
    for cname, py in [("mcrt_grid_desc", M.GridDesc), ("mcrt_opacity_desc", M.OpacityDesc),
                      ("mcrt_solve_params", M.SolveParams), ("mcrt_result", M.Result)]:
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", txt).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            parts = [x.strip() for x in decl.split(",")]
            fields.append(parts[0].split()[-1].lstrip("*"))
            fields.extend(x.lstrip("*") for x in parts[1:])
        assert [f[0] for f in py._fields_] == fields, cname


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcrt.so not built")
def test_default_params_and_error_string_need_no_device():
    from paper_2110_15640_amd import mcrt as M
    p = M.default_params()
    assert p.rr_threshold == 1e-3 and p.rr_survive == 0.1 and p.emis_bias == 0.5
    assert p.tau_vert_max == 30.0 and p.max_events == 1000000 and p.n_b == 256 and p.n_alpha == 360
    assert isinstance(M.load().mcrt_last_error(), bytes)


def _c_layout(structs):
    """sizeof and offsetof of every field, from the header compiled by gcc."""
    import shutil
    import subprocess
    import tempfile
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mcrt.h"', "int main(void) {"]
    for cname, fields in structs:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines))
        subprocess.check_call([gcc, "-I", os.path.dirname(HEADER), "-o", exe, src])
        out = subprocess.check_output([exe]).decode()
    res = {}
    for ln in out.splitlines():
        a, b, c = ln.split()
        res[(a, b)] = int(c)
    return res


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcrt.so not built")
def test_binding_struct_offsets_and_sizes_match_the_c_compiler():
    """Beyond the field names: every ctypes offset and struct size equals what
    a C compiler makes of the header, so no field has a mismatched type."""
    from paper_2110_15640_amd import mcrt as M
    pairs = [("mcrt_grid_desc", M.GridDesc), ("mcrt_opacity_desc", M.OpacityDesc),
             ("mcrt_solve_params", M.SolveParams), ("mcrt_result", M.Result), ("mcrt_batch_item", M.BatchItem)]
    lay = _c_layout([(c, [f[0] for f in py._fields_]) for c, py in pairs])
    for cname, py in pairs:
        assert lay[(cname, "size")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert lay[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def _prototypes():
    """name -> list of parameter declarations, from the header's prototypes."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"\b(?:int|void|uint64_t|const char\*)\s+(mcrt_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", txt):
        args = [a.strip() for a in m.group(2).split(",") if a.strip() and a.strip() != "void"]
        out[m.group(1)] = args
    return out


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmcrt.so not built")
def test_binding_argtypes_match_header_prototypes():
    """Every function the binding declares takes as many arguments as its C
    prototype; the uploads take the caller's stream before the id."""
    from paper_2110_15640_amd import mcrt as M
    L = M.load()
    protos = _prototypes()
    assert set(protos) == set(declared_functions())
    checked = 0
    for name, args in protos.items():
        at = getattr(L, name).argtypes
        if at is None:
            continue
        assert len(at) == len(args), (name, args)
        checked += 1
    assert checked >= 15
    for name in ("mcrt_grid_upload", "mcrt_opacity_upload"):
        assert protos[name][2].replace(" ", "") == "void*stream", protos[name]
    assert protos["mcrt_solve_noalloc"][1].replace(" ", "") == "int32_tmode"
