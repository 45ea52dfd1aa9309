"""The ctypes mirrors of the structs that cross the C ABI have exactly the
layout a C compiler gives the declarations in include/clb.h: the same
fields in the same order, the same offset and size of every field, and the
same total size.  A small C program built with gcc prints the C side; no GPU
and no library are involved."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")

clb = pytest.importorskip("paper_1603_01955_amd.clb")
clb3d = pytest.importorskip("paper_1603_01955_amd.clb3d")

MIRRORS = {"clb_params": clb.clb_params, "clb_derived": clb.clb_derived, "clb3_params": clb3d.clb3_params}


def _header_fields(name):
    """Field names of `typedef struct name { ... } name;` in declaration order."""
    text = "".join(open(os.path.join(INCLUDE, h)).read() for h in sorted(os.listdir(INCLUDE)) if h.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    m = re.search(r"typedef\s+struct\s+%s\s*\{(.*?)\}\s*%s\s*;" % (name, name), text, flags=re.S)
    assert m, name
    fields = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        # "double rho0, ux0, uy0" -> three fields
        head, _, rest = decl.partition(" ")
        fields += [f.strip() for f in rest.split(",")]
    return fields


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "clb3d.h"', "int main(void) {"]
    for name in MIRRORS:
        lines.append('  printf("%s SIZE %%zu 0\\n", sizeof(%s));' % (name, name))
        for f in _header_fields(name):
            lines.append('  printf("%s %s %%zu %%zu\\n", offsetof(%s, %s), sizeof(((%s*)0)->%s));'
                         % (name, f, name, f, name, f))
    lines += ["  return 0;", "}"]
    d = tmp_path_factory.mktemp("layout")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", INCLUDE, str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    layout = {}
    for line in out.splitlines():
        struct, field, off, size = line.split()
        layout.setdefault(struct, {})[field] = (int(off), int(size))
    return layout


@pytest.mark.parametrize("name", sorted(MIRRORS))
def test_mirror_has_the_header_fields_in_order(name):
    assert [f[0] for f in MIRRORS[name]._fields_] == _header_fields(name)


@pytest.mark.parametrize("name", sorted(MIRRORS))
def test_mirror_offsets_sizes_and_total_size(name, c_layout):
    py = MIRRORS[name]
    c = c_layout[name]
    assert ctypes.sizeof(py) == c["SIZE"][0]
    for field, ctype in py._fields_:
        off, size = c[field]
        assert getattr(py, field).offset == off, field
        assert ctypes.sizeof(ctype) == size, field
