"""Host-side checks of the C ABI (no GPU needed): the built library loads,
exports every function include/ecmc.h declares, and sizes workspaces."""
import ctypes
import os
import re

import pytest

import paper_2004_11040_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions(header="ecmc.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(ecmc_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_every_header_has_a_library():
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == ["ecmc.h", "ecmc_probe.h"]


@pytest.mark.parametrize("header,exports,path", [
    ("ecmc.h", pkg.EXPORTS, pkg.LIB_PATH),
    ("ecmc_probe.h", pkg.PROBE_EXPORTS, pkg.PROBE_LIB_PATH),
])
def test_library_exports_every_declared_symbol(header, exports, path):
    assert _declared_functions(header) == sorted(exports)
    lib = ctypes.CDLL(path)
    for name in _declared_functions(header):
        assert hasattr(lib, name), name


def test_workspace_bytes_host_only():
    n = 4096
    L = 135.58
    b = pkg.workspace_bytes(n, 1.0, L, 0, 64, 1024)
    assert b > 0 and b % 256 == 0
    # grows with chains and log capacity
    assert pkg.workspace_bytes(n, 1.0, L, 0, 128, 1024) > b
    assert pkg.workspace_bytes(n, 1.0, L, 0, 64, 4096) > b
    # the FP32-mixed form filters in registers: same workspace
    assert pkg.workspace_bytes(n, 1.0, L, 0, 64, 1024, pkg.FP32_MIXED) == b


@pytest.mark.parametrize("args", [
    (1, 1.0, 50.0, 0, 1, 1),          # n < 2
    (100, 0.0, 50.0, 0, 1, 1),        # sigma <= 0
    (100, 1.0, -1.0, 0, 1, 1),        # box <= 0
    (100, 1.0, 50.0, 30, 1, 1),       # cell narrower than 2 sigma
    (100, 1.0, 50.0, 5, 1, 1),        # cell wider than 2 sqrt(2) sigma
    (100, 1.0, 8.0, 0, 1, 1),         # fewer than 5 cells per side
    (100, 1.0, 50.0, 0, 0, 1),        # no chains
    (100, 1.0, 50.0, 0, 1, 0),        # no log
    (10000, 1.0, 50.0, 0, 1, 1),      # more disks than slots
])
def test_workspace_bytes_rejects(args):
    assert pkg.workspace_bytes(*args) == pkg.EINVAL


def test_workspace_flags_rejected():
    assert pkg.workspace_bytes(100, 1.0, 50.0, 0, 1, 1, flags=8) == pkg.EINVAL


@pytest.mark.parametrize("cname,pyclass", [("ecmc_stats_t", pkg.Stats), ("ecmc_batch_info_t", pkg.BatchInfo)])
def test_struct_layouts_agree_with_the_header(cname, pyclass, tmp_path):
    """Compile the header with the host C compiler and compare the size and
    every field offset of the result structs with the binding's ctypes view."""
    import subprocess
    fields = [n for n, _ in pyclass._fields_]
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ecmc.h"', "int main(void) {",
             f'printf("size %zu\\n", sizeof({cname}));']
    lines += [f'printf("{f} %zu\\n", offsetof({cname}, {f}));' for f in fields]
    lines += ["return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    assert int(out["size"]) == ctypes.sizeof(pyclass)
    for f in fields:
        assert int(out[f]) == getattr(pyclass, f).offset, f


def test_option_and_feature_constants_agree_with_the_header():
    """Every ECMC_OPT_*, ECMC_FEAT_* and ECMC_NEIGHBOURS_* value the header
    defines is the binding's constant of the same name, and the binding has
    no option the header lacks."""
    src = open(os.path.join(ROOT, "include", "ecmc.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in
            re.finditer(r"#define\s+ECMC_((?:OPT|FEAT|NEIGHBOURS)_[A-Z0-9_]+)\s+(\d+)u?\b", src)}
    assert len(defs) > 20
    for name, value in defs.items():
        assert getattr(pkg, name) == value, name
    opts = {n for n in dir(pkg) if n.startswith("OPT_")}
    assert opts == {n for n in defs if n.startswith("OPT_")}
