"""The binding's view of the C-ABI agrees with include/abd.h (host only, no
GPU): every structure the binding passes has the size and field offsets the
C compiler gives it, and every entry point's return and argument types in
the binding are those of the header's prototype, in order.  A field added
to a header structure or an argument added to a prototype without the same
change in the binding fails here instead of passing garbage to the
library."""
import ctypes as C
import os
import re
import shutil
import subprocess

import pytest

from paper_2605_15875_amd import abd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abd.h")

STRUCTS = {"abd_params": abd.Params, "abd_tuning": abd.Tuning,
           "abd_admm_params": abd.AdmmParams,
           "abd_admm_report": abd.AdmmReport, "abd_stats": abd.Stats,
           "abd_balance": abd.BalanceState}
OPAQUE = ("abd_ctx", "abd_batch", "abd_consensus")
SCALARS = {"double": C.c_double, "int32_t": C.c_int32, "int64_t": C.c_int64,
           "size_t": C.c_size_t, "int": C.c_int, "char": C.c_char}


def header_text():
    t = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return "\n".join(l for l in t.splitlines() if not l.strip().startswith("#"))


def prototypes():
    """name -> (return type, [parameter declarations]) of every entry point"""
    out = {}
    for m in re.finditer(r"([A-Za-z_][\w \t\*]*?)\b(abd_[a-z_]+)\s*\(([^;{]*?)\)\s*;",
                         header_text()):
        params = [p.strip() for p in m.group(3).split(",")]
        if params == ["void"] or params == [""]:
            params = []
        out[m.group(2)] = (m.group(1).strip(), params)
    return out


def ctype_of(decl, named=True):
    """ctypes type of a C declaration ('const double* x', 'abd_ctx** out')"""
    d = re.sub(r"\bconst\b", " ", decl)
    stars = d.count("*")
    words = d.replace("*", " ").split()
    base = words[0]
    if named:
        assert len(words) == 2, decl
    if base in OPAQUE:
        assert stars >= 1, decl
        t, stars = C.c_void_p, stars - 1
    elif base == "void":
        if stars == 0:
            return None
        t, stars = C.c_void_p, stars - 1
    elif base == "char" and stars == 1:
        t, stars = C.c_char_p, 0
    elif base in STRUCTS:
        t = STRUCTS[base]
    else:
        t = SCALARS[base]
    for _ in range(stars):
        t = C.POINTER(t)
    return t


def test_header_parse_finds_every_export():
    assert set(prototypes()) == set(abd.EXPORTS)


def test_entry_point_types_match_the_header():
    L = abd.lib()
    for name, (ret, params) in prototypes().items():
        f = getattr(L, name)
        assert f.restype == ctype_of(ret, named=False), name
        want = [ctype_of(p) for p in params]
        assert list(f.argtypes) == want, (name, params, f.argtypes)


def test_structure_layouts_match_the_compiler(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "abd.h"',
           "int main(void) {"]
    for cname, cls in STRUCTS.items():
        src.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            src.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    src += ["return 0;", "}"]
    c_file = tmp_path / "layout.c"
    c_file.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I",
                    os.path.join(ROOT, "include"), str(c_file), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True,
                         text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            s, f, v = line.split()
            got[(s, f)] = int(v)
    for cname, cls in STRUCTS.items():
        assert C.sizeof(cls) == got[(cname, "sizeof")], cname
        for f, _ in cls._fields_:
            assert getattr(cls, f).offset == got[(cname, f)], (cname, f)


def test_structures_have_every_header_field():
    """each header structure's field names, in order, are the binding's
    (the offsets above cannot see a field the binding lacks at the end)"""
    t = header_text()
    for cname, cls in STRUCTS.items():
        body = re.search(r"typedef struct " + cname + r"\s*\{(.*?)\}\s*" + cname + ";",
                         t, flags=re.S).group(1)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            first, *rest = [d.strip() for d in decl.split(",")]
            names.append(re.sub(r"\[.*\]", "", first.split()[-1]).lstrip("*"))
            names += [re.sub(r"\[.*\]", "", r).lstrip("*") for r in rest]
        assert names == [f for f, _ in cls._fields_], (cname, names)
