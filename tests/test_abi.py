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
           ("uhm_block_desc", binding.BlockDesc), ("uhm_coupling_desc", binding.CouplingDesc))


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
    for dt, st in ((binding.BLOCK_DTYPE, binding.BlockDesc), (binding.COUPLING_DTYPE, binding.CouplingDesc)):
        assert dt.itemsize == ctypes.sizeof(st)
        for f, _ in st._fields_:
            assert dt.fields[f][1] == getattr(st, f).offset


def test_construction_entry_points_validate_before_any_device_work():
    """uhm_aca and uhm_kernel_blocks check their scalar arguments on the host and return
    before touching the device, so these calls run without a GPU."""
    import ctypes
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libuhm.so is not built")
    lib = binding.load_library()
    null = ctypes.c_void_p(0)

    def aca(nblocks=0, max_rows=64, max_cap=16, eps=1e-6, npoints=10, kappa=1.0):
        return lib.uhm_aca(null, npoints, kappa, 1.0, null, nblocks, max_rows, max_cap, eps,
                           null, 0, null, 0, null, 0, null, null, null)

    assert aca() == binding.UHM_OK                       # nothing to do
    assert aca(max_rows=0) == binding.UHM_EINVAL
    assert aca(max_rows=65537) == binding.UHM_EINVAL
    assert aca(max_cap=0) == binding.UHM_EINVAL
    assert aca(max_cap=1025) == binding.UHM_EINVAL
    assert aca(eps=-1.0) == binding.UHM_EINVAL
    assert aca(eps=float("nan")) == binding.UHM_EINVAL
    assert aca(kappa=float("inf")) == binding.UHM_EINVAL
    assert aca(npoints=-1) == binding.UHM_EINVAL
    assert aca(nblocks=3) == binding.UHM_EINVAL          # null pointers with blocks to do
    assert b"null pointer" in lib.uhm_last_error()

    def dense(nblocks=0, npoints=10, D_len=0):
        return lib.uhm_kernel_blocks(null, npoints, 1.0, 1.0, null, nblocks, null, D_len, null, null)

    assert dense() == binding.UHM_OK
    assert dense(npoints=-5) == binding.UHM_EINVAL
    assert dense(D_len=-1) == binding.UHM_EINVAL
    assert dense(nblocks=2) == binding.UHM_EINVAL
