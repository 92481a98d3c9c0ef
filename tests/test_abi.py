"""Host-side checks of the C-ABI library (CPU only, no device calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1609_06068_amd import cdcs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "cdcs.h")).read()
    return sorted(set(re.findall(r"^(?:cdcs_status|const char \*)\s*(cdcs_\w+)\(", src, flags=re.M)))


def test_header_declarations_match_binding_list():
    assert _declared_symbols() == sorted(cdcs.EXPORTS)


def test_library_loads_and_exports_every_declared_symbol():
    if not os.path.exists(cdcs.LIB_PATH):
        pytest.skip("libcdcs.so not built")
    lib = ctypes.CDLL(cdcs.LIB_PATH)
    for name in _declared_symbols():
        assert hasattr(lib, name), name
    L = cdcs.load_library()
    assert L.cdcs_last_error() is not None


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(cdcs.CdcsLibraryMissing):
        cdcs._lib_backup = cdcs._lib
        try:
            cdcs._lib = None
            cdcs.load_library(str(tmp_path / "nope.so"))
        finally:
            cdcs._lib = cdcs._lib_backup


def test_packing_roundtrip():
    rng = np.random.default_rng(0)
    blocks = []
    for s in [1, 3, 5]:
        R = rng.standard_normal((s, s))
        blocks.append(R + R.T)
    packed = cdcs.pack_blocks(blocks)
    assert packed.shape[0] == 1 + 6 + 15
    back = cdcs.unpack_blocks(packed, [1, 3, 5])
    for a, b in zip(blocks, back):
        assert np.array_equal(a, b)
    # slot (a, b) of a block sits at a(a+1)/2 + b
    assert packed[1 + (2 * 3 // 2 + 1)] == blocks[1][2, 1]


# C structs of include/cdcs.h and their ctypes mirrors in the binding.
_STRUCTS = {
    "cdcs_pattern": cdcs._Pattern, "cdcs_cliques": cdcs._Cliques, "cdcs_constraints": cdcs._Constraints,
    "cdcs_options": cdcs._Options, "cdcs_info": cdcs._Info, "cdcs_state": cdcs._State,
    "cdcs_problem": cdcs._Problem, "cdcs_instance_info": cdcs._InstanceInfo, "cdcs_tuning": cdcs._Tuning,
    "cdcs_sizes": cdcs._Sizes, "cdcs_vcones": cdcs._Vcones, "cdcs_hsde_state": cdcs._HsdeState,
    "cdcs_hsde_info": cdcs._HsdeInfo,
}


def test_struct_layouts_match_the_header(tmp_path):
    """Compile a host program against include/cdcs.h with g++ and compare every
    struct's size and field offsets with the ctypes definitions."""
    import shutil
    import subprocess
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("g++ or the ROCm headers are not available")
    lines = ['#include <cstdio>', '#include <cstddef>', '#include "cdcs.h"', "int main() {"]
    for cname, py in _STRUCTS.items():
        lines.append(f'  std::printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  std::printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.cpp"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", "/opt/rocm/include", str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in _STRUCTS.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
