"""CPU checks of the C ABI: the library loads and exports every entry point
declared in include/pfe.h; the ctypes structures match the header's layout."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfe.h")
LIB = os.path.join(ROOT, "paper_1612_06496_amd", "libpfe.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pfe_[A-Za-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pfe_build_graph", "pfe_init", "pfe_step", "pfe_solve"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpfe.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpfe.so not built")
def test_status_strings_and_binding_signatures():
    from paper_1612_06496_amd import _lib as L
    assert set(L.SIGNATURES) == set(declared_functions())
    assert L.lib.pfe_status_string(L.PFE_E_RANK).decode().startswith("rank")
    assert L.lib.pfe_status_string(L.PFE_OK).decode() == "ok"
    # null-argument paths return PFE_E_ARG without touching a GPU
    assert L.lib.pfe_build_graph(None, None, None) == L.PFE_E_ARG
    assert L.lib.pfe_step(None, 0, None) == L.PFE_E_ARG
    assert L.lib.pfe_graph_info(None, None, None, None) == L.PFE_E_ARG


def test_struct_layouts_match_header(tmp_path):
    """Every ctypes field offset equals offsetof() of the C header, compiled with gcc."""
    import shutil
    import subprocess
    from paper_1612_06496_amd import _lib as L
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = [L.pfe_graph_desc, L.pfe_params, L.pfe_step_info, L.pfe_monitors, L.pfe_tune_result]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pfe.h"', "int main(void){"]
    for st in structs:
        cname = st.__name__
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for fname, _ in st._fields_:
            cf = "lambda" if fname == "lambda_" else fname
            lines.append(f'printf("%zu\\n", offsetof({cname}, {cf}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = []
    for st in structs:
        want.append(ctypes.sizeof(st))
        for fname, _ in st._fields_:
            want.append(getattr(st, fname).offset)
    assert got == want


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpfe.so not built")
def test_argument_checks_of_later_entry_points_need_no_gpu():
    """Argument validation of the Stage II, FSAI, k-means and allocator entry
    points happens on the host before any device call."""
    import ctypes as C
    from paper_1612_06496_amd import _lib as L
    lib = L.lib
    assert lib.pfe_split_bregman(None, 3, None) == L.PFE_E_ARG
    assert lib.pfe_set_fsai(None) == L.PFE_E_ARG
    it = C.c_int32()
    # k-means: null pointers, K above 256, d above 32, no iteration
    assert lib.pfe_kmeans(None, 10, 4, L.PFE_FP32, None, 3, 10, None, None, C.byref(it), None) == L.PFE_E_ARG
    dummy = C.c_void_p(1)
    assert lib.pfe_kmeans(dummy, 10, 4, L.PFE_FP32, dummy, 300, 10, dummy, dummy, None, None) == L.PFE_E_ARG
    assert lib.pfe_kmeans(dummy, 10, 40, L.PFE_FP32, dummy, 3, 10, dummy, dummy, None, None) == L.PFE_E_ARG
    assert lib.pfe_kmeans(dummy, 10, 4, L.PFE_FP32, dummy, 3, 0, dummy, dummy, None, None) == L.PFE_E_ARG
    assert lib.pfe_kmeans(dummy, 10, 4, 7, dummy, 3, 10, dummy, dummy, None, None) == L.PFE_E_ARG
    # allocator: both functions or neither; no live allocation in a fresh process
    assert lib.pfe_live_allocations() == 0
    assert lib.pfe_set_allocator(dummy, None, None) == L.PFE_E_ARG
    assert lib.pfe_set_allocator(None, None, None) == L.PFE_OK


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpfe.so not built")
def test_network_file_format_is_checked_on_the_host(tmp_path):
    """pfe_mpnn_load rejects a missing file, a wrong magic, a wrong count, a
    truncated or over-long file and non-finite values before taking device
    memory (so without a GPU)."""
    import ctypes as C
    import struct
    import numpy as np
    from paper_1612_06496_amd import _lib as L
    h = C.c_void_p()
    n = L.PFE_MPNN_NPARAMS
    good = np.zeros(n, dtype="<f4")
    cases = {
        "missing": None,
        "magic": b"XXXXXXXX" + struct.pack("<I", n) + good.tobytes(),
        "count": b"PFEMPNN1" + struct.pack("<I", n - 1) + good[:-1].tobytes(),
        "short": b"PFEMPNN1" + struct.pack("<I", n) + good[:-3].tobytes(),
        "long": b"PFEMPNN1" + struct.pack("<I", n) + good.tobytes() + b"\0",
        "nan": b"PFEMPNN1" + struct.pack("<I", n) + np.full(n, np.nan, dtype="<f4").tobytes(),
    }
    for name, blob in cases.items():
        path = tmp_path / f"{name}.bin"
        if blob is not None:
            path.write_bytes(blob)
        assert L.lib.pfe_mpnn_load(str(path).encode(), C.byref(h)) == L.PFE_E_ARG, name
        assert not h.value


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpfe.so not built")
def test_binding_module_imports():
    """The Python binding loads without a GPU (its calls need one)."""
    import importlib
    mod = importlib.import_module("paper_1612_06496_amd.solver")
    for name in ("Graph", "Solver", "Mpnn", "kmeans", "close_all"):
        assert hasattr(mod, name)
