"""The C-ABI library loads and exports every entry point include/uhm.h declares (no GPU)."""
import os
import re

import pytest

from paper_2405_15573_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "uhm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(uhm_[a-z_0-9]+)\s*\(", text)))


def test_header_lists_the_binding_exports():
    assert set(declared_functions()) == set(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libuhm.so is not built")
    lib = binding.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.uhm_version() >= 1
    assert lib.uhm_strerror(binding.UHM_EINVAL) == b"invalid argument"


STRUCTS = (("uhm_host_operator", binding.HostOperator), ("uhm_host_hmatrix", binding.HostHMatrix),
           ("uhm_op_info", binding.OpInfo), ("uhm_gmres_opts", binding.GmresOpts), ("uhm_gmres_info", binding.GmresInfo),
           ("uhm_block_desc", binding.BlockDesc))


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes field offset equals offsetof() of the C struct compiled from uhm.h."""
    import ctypes
    import subprocess
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "uhm.h"', "int main(void) {"]
    for cname, py in STRUCTS:
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.split("\n") if l)
    for cname, py in STRUCTS:
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


def test_block_record_matches_struct():
    import ctypes
    assert binding.BLOCK_DTYPE.itemsize == ctypes.sizeof(binding.BlockDesc)
    for f, _ in binding.BlockDesc._fields_:
        assert binding.BLOCK_DTYPE.fields[f][1] == getattr(binding.BlockDesc, f).offset
