"""The binding's ctypes structures match the C header field by field (offset and size), every
structure the header declares has a binding counterpart, and every declared function is bound
with the header's number of parameters.  A C program built
from the header with the host compiler prints the layout; no GPU is involved."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smoothgemm.h")


def _binding_structs():
    import paper_2605_29752_amd as sg
    return {n: c for n, c in vars(sg).items()
            if isinstance(c, type) and issubclass(c, ctypes.Structure) and n.startswith("sg_")}


def _c_layout(structs, tmp_path):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "smoothgemm.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for f in cls._fields_:
            lines.append('printf("%s.%s %%zu %%zu\\n", offsetof(%s, %s), sizeof(((%s*)0)->%s));'
                         % (name, f[0], name, f[0], name, f[0]))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    res = {}
    for ln in out.splitlines():
        key, a, b = ln.split()
        res[key] = int(b) if a == "size" else (int(a), int(b))
    return res


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_ctypes_structs_match_header(tmp_path):
    structs = _binding_structs()
    c = _c_layout(structs, tmp_path)
    for name, cls in structs.items():
        assert c[name] == ctypes.sizeof(cls), "%s: C size %d, ctypes %d" % (name, c[name], ctypes.sizeof(cls))
        for f in cls._fields_:
            fd = getattr(cls, f[0])
            assert c["%s.%s" % (name, f[0])] == (fd.offset, fd.size), "%s.%s layout differs" % (name, f[0])


def _header_fields():
    """{struct name: [field names in declaration order]} parsed from the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for name, body in re.findall(r"typedef struct (sg_\w+)\s*\{(.*?)\}\s*\1\s*;", text, flags=re.S):
        names = []
        for decl in body.split(";"):
            for part in decl.split(","):
                m = re.search(r"(\w+)\s*(\[[^\]]*\])?\s*$", part.strip())
                if m:
                    names.append(m.group(1))
        out[name] = names
    return out


def test_every_header_struct_is_bound_field_for_field():
    declared = _header_fields()
    bound = _binding_structs()
    assert set(declared) <= set(bound), "structures without a binding: %s" % sorted(set(declared) - set(bound))
    for name, fields in declared.items():
        assert [f[0] for f in bound[name]._fields_] == fields, "%s: fields differ from the header" % name


def _header_prototypes():
    """{function name: parameter count} of every prototype in the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    text = re.sub(r"#[^\n]*", "", text)
    out = {}
    for m in re.finditer(r"\b(\w+)\s*\(([^;{}()]*)\)\s*;", text):
        name, params = m.group(1), m.group(2).strip()
        if name.startswith(("sg_", "gemm_")) and not name.endswith("_t"):
            out[name] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_signatures_match_header_arity():
    import paper_2605_29752_amd as sg
    protos = _header_prototypes()
    sigs = sg._SIGS
    assert len(protos) > 40
    missing = sorted(set(sigs) - set(protos))
    assert not missing, "bound but not declared: %s" % missing
    unbound = sorted(set(protos) - set(sigs))
    assert not unbound, "declared but not bound: %s" % unbound
    for name, (_, args) in sigs.items():
        assert len(args) == protos[name], "%s: header has %d parameters, binding %d" % (name, protos[name], len(args))
